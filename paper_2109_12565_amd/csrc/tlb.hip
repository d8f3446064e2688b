// Host side of the C ABI declared in include/tlb.h: parameter checks, device
// memory, launch geometry, and the step / observable / export sequences.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "tlb.h"
#include "droplets.hpp"
#include "launch.hpp"
#include "lb_kernels.hpp"
#include "lb_reduce.hpp"

namespace {

thread_local char g_init_error[512];

}  // namespace

struct tlb_handle {
  tlb_params p{};
  int device = 0;                  // HIP device current at tlb_init
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool external = false;           // buf, partials, obs, t_bottom, solid, link in a
                                   // caller's workspace (tlb_init_external)
  // the adjoint's second stream (segment recompute beside the reverse
  // sweep, default priority) and its events, created on first use
  hipStream_t side = nullptr;
  hipEvent_t ev_side[2] = {nullptr, nullptr};   // recompute of a segment done
  hipEvent_t ev_main[3] = {nullptr, nullptr, nullptr};  // reverse sweep done, start
  int pitch = 0;
  long long pop_stride = 0;
  size_t elem = 0;                 // bytes per stored population value
  void* buf[2] = {nullptr, nullptr};
  int cur = 0;                     // buf[cur] = f*(t); buf[1-cur] = f*(t-1) or f(0)
  int64_t t = 0;
  bool has_solid = false;
  uint16_t* link = nullptr;
  uint8_t* solid = nullptr;
  void* t_bottom = nullptr;        // C-typed copy of the bottom temperature
  double* partials = nullptr;
  double* obs = nullptr;           // [6]
  double* fields = nullptr;        // [7][ly][lx], allocated on first use
  double* rows = nullptr;          // [2][ly] row averages, allocated on first use
  // droplet detection, allocated on first use
  int32_t* drop_nodes = nullptr;   // [3][ly*lx] parent, root number, label
  int32_t* drop_tiles = nullptr;   // [tiles + 1] roots per tile, offsets
  int* drop_error = nullptr;
  double* drop_tb = nullptr;       // [lx] FP64 bottom temperature
  void* drop_acc = nullptr;        // per droplet: sums, root, output record
  size_t drop_acc_cap = 0;         // droplets drop_acc has room for
  double* export_buf = nullptr;    // [27][ly][lx], allocated on first use
  double n_fluid = 0, n_top = 0;
  std::vector<uint8_t> host_solid;  // [ly*lx] solid flags (host copy)
  std::vector<double> host_tb;      // [lx] bottom wall temperature (host copy)
  double dtdy_sum = 0;             // fluid-node sum of the central dT/dy
  int64_t obs_t = -1;              // time of the observable sums in partials
  tlbh::Geometry launch{};
  bool tau_one = false;            // tau = tau_g = 1: equilibria path
  // adjoint tape (flat walls, FP64 / FP32 storage)
  void* ckpt = nullptr;            // checkpoints of f*, ckpt_cap states
  size_t ckpt_cap = 0;
  void* tape = nullptr;            // recomputed states of one segment
  size_t tape_cap = 0;
  void* mtape = nullptr;           // tau = 1: moments of the pulled state of each
  size_t mtape_cap = 0;            // taped step (or of one segment), 5 planes each
  void* adj = nullptr;             // AdjointWork planes
  double* adj_scalars = nullptr;   // grad [lx] + loss terms [loss_cap]
  size_t loss_cap = 0;
  int64_t taped_steps = 0;
  int ckpt_every = 0;
  bool tape_valid = false;
  char err[512] = {0};
};

namespace {

int fail(tlb_handle* h, int code, const char* fmt, ...) {
  char* dst = h ? h->err : g_init_error;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return code;
}

#define TLB_HIP(h, expr)                                                           \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail((h), TLB_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool is_fp64(const tlb_handle* h) { return h->p.precision == TLB_FP64; }

size_t storage_bytes(int precision) {
  return precision == TLB_FP64 ? sizeof(double) : (precision == TLB_FP32 ? sizeof(float) : 2);
}

// Size of a population buffer in stored planes: 27, plus for the 16-bit
// floating deviations three FP32 rest planes (two 16-bit planes each).
size_t buffer_planes(int precision) {
  return precision == TLB_FP16_DEV || precision == TLB_BF16_DEV ? 27 + 3 * 2 : 27;
}

// Call f with a value of the storage policy type of the handle's precision.
template <class F>
void with_storage(int precision, F&& f) {
  switch (precision) {
    case TLB_FP64: f(tlbk::Store<double>{}); break;
    case TLB_FP32: f(tlbk::Store<float>{}); break;
    case TLB_FP16_DEV: f(tlbk::StoreF16Dev{}); break;
    case TLB_BF16_DEV: f(tlbk::StoreBF16Dev{}); break;
    default: f(tlbk::StoreFix16Dev{}); break;
  }
}

// Launch geometry: 256-wide strips for wide lattices, 64-wide otherwise.
// The row-chunk height is chosen so that the grid holds a whole number of
// blocks per compute unit, `target` of them (at most what the kernel's
// occupancy allows): the step is a single wave of resident blocks, and an
// uneven count leaves some CUs with one block more than others. Storages of
// 4 bytes and more are bandwidth bound and prefer fewer, taller chunks (less
// halo re-read): 16 wavefronts per CU (4 blocks of 256); the 16-bit
// storages are latency bound and prefer 20. Rows are kept in [5, 65] with
// rows + 4 a multiple of 3 (the row loop is unrolled three times);
// p.rows > 0 sets the row count.
tlbh::Geometry choose_launch(const tlb_params& p, size_t buffer_bytes, bool solid, bool tau_one) {
  tlbh::Geometry l;
  const int lx = p.lx, ly = p.ly;
  // 32-bit byte offsets address the whole population buffer below 4 GiB;
  // TLB_LAUNCH_WIDE_OFFSETS selects the 64-bit variant at any size.
  l.wide = buffer_bytes > 0xFFFFFFFFull || (p.launch_flags & TLB_LAUNCH_WIDE_OFFSETS) != 0;
  l.bx = (lx >= 2048 || l.wide) ? 256 : 64;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int per_cu = 1;
  with_storage(p.precision, [&](auto st) {
    per_cu = tlbh::Launcher<decltype(st)>::blocks_per_cu(l.bx, l.wide, solid, tau_one);
  });
  const int target_waves = storage_bytes(p.precision) >= 4 ? 16 : 20;
  const int target = std::max(1, std::min(per_cu, target_waves / (l.bx / 64)));
  const long long strips = (lx + l.bx - 1) / l.bx;
  long long rows = (ly * strips + (long long)cus * target - 1) / ((long long)cus * target);
  // Floor of 5 rows: each chunk pulls 4 extra rows, and lattices too small
  // to give every CU its target waves (1024 x 512: 2 rows) trade occupancy
  // against that overhead best there (measured 36.6 us per step at 5 rows,
  // 39.0 at 2, 41.0 at 8, 48.0 at 11).
  rows = rows < 5 ? 5 : (rows > 65 ? 65 : rows);
  while ((rows + 4) % 3) ++rows;
  if (p.rows > 0) rows = p.rows;
  l.rows = (int)(rows < ly ? rows : ly);
  l.grid = dim3((unsigned)strips, (unsigned)((ly + l.rows - 1) / l.rows), 1);

  // Fused two-step kernel: tau = tau_g = 1, any storage but fixed point, 32-bit
  // offsets. Its strips overlap by kStep2Halo columns and its
  // chunks recompute 5 rows of the first step on each side, so it pays
  // where the grid fills every CU once: one block per resident slot.
  // TLB_FUSED_ALWAYS selects it wherever it applies (FP64 included),
  // TLB_FUSED_NEVER never.
  const bool eligible = tau_one && !l.wide && p.precision != TLB_FIX16_DEV;
  if (eligible && p.fused != TLB_FUSED_NEVER) {
    // Geometry for blocks of `lanes` lanes: strips of at most lanes -
    // kStep2Halo stored columns, and at most one block per resident slot (a
    // second, partial wave of blocks would take as long as the first).
    struct Fused {
      int per_cu = 0, strip = 0;
      long long strips = 1, rows = 1;
    };
    auto fused_geometry = [&](int lanes) {
      Fused g;
      with_storage(p.precision, [&](auto st) {
        g.per_cu = tlbh::Launcher<decltype(st)>::step2_blocks_per_cu(solid, lanes);
      });
      int max_strip = lanes - tlbh::kStep2Halo;
      if (p.fused_strip > 0) max_strip = std::min(max_strip, (int)p.fused_strip);
      g.strips = (lx + max_strip - 1) / max_strip;
      g.strip = (int)((lx + g.strips - 1) / g.strips);
      const long long slots = (long long)cus * std::max(g.per_cu, 1);
      const long long max_chunks = std::max(1LL, slots / g.strips);
      g.rows = (ly + max_chunks - 1) / max_chunks;
      return g;
    };
    const Fused wide = fused_geometry(tlbh::kStep2Lanes);
    // Narrow blocks where wide ones would leave chunks of fewer than 16 rows:
    // a block's time is then mostly its chain of first-level halo rows, and
    // twice as many resident narrow blocks take shorter chunks (FP32 per
    // fused launch, 256 / 128 lanes: 1024 x 512 54.8 / 49.5 us, 1024 x 64
    // 28.7 / 27.0, 128 x 64 24.8 / 23.5; 4096 x 2048 with 69-row chunks
    // 527 / 596, FP16 deviations 494 / 512). Also where wide blocks do not
    // fit twice per CU (FP64: 158 KB of LDS), since one resident block per
    // CU does not pay (FP64 per step, single / fused 256 / fused 128 lanes:
    // 4096 x 2048 751.7 / 769.0 / 677.5 us, 1024 x 512 64.8 / 63.0 / 52.2).
    const bool narrow = p.fused_lanes == tlbh::kStep2LanesNarrow ||
                        (p.fused_lanes == 0 && (wide.rows < 16 || wide.per_cu < 2));
    const Fused g2 = narrow ? fused_geometry(tlbh::kStep2LanesNarrow) : wide;
    const int per_cu2 = g2.per_cu;
    const long long strips2 = g2.strips;
    const int strip2 = g2.strip;
    long long rows2 = g2.rows;
    // with at least two resident blocks per CU it pays at every lattice size
    // measured, the chunk height being the one that fills the slots once
    // (FP32 per step, fused / single: 128 x 64 12.7 / 20.1 us, 1024 x 64
    // 14.9 / 20.7, 1024 x 256 20.9 / 28.0, 1024 x 512 28.1 / 36.8, 2048 x
    // 1024 68.7 / 101.5, 4096 x 2048 263 / 377, all in 256-lane blocks; the
    // 16-bit storages equal or faster); taller chunks in a second wave of
    // blocks cost more than the halo rows they save.
    const bool pays = per_cu2 >= 2;
    if (per_cu2 > 0 && (pays || p.fused == TLB_FUSED_ALWAYS)) {
      if (p.fused_rows > 0) rows2 = p.fused_rows;
      l.rows2 = (int)(rows2 < ly ? rows2 : ly);
      l.lanes2 = narrow ? tlbh::kStep2LanesNarrow : tlbh::kStep2Lanes;
      l.strip2 = strip2;
      l.grid2 = dim3((unsigned)strips2, (unsigned)((ly + l.rows2 - 1) / l.rows2), 1);
    }
  }
  return l;
}

tlbh::Device device_view(const tlb_handle* h, double* fields = nullptr,
                         double* partials = nullptr) {
  tlbh::Device d;
  d.p = &h->p;
  d.stream = h->stream;
  d.geo = h->launch;
  d.pitch = h->pitch;
  d.pop_stride = h->pop_stride;
  d.has_solid = h->has_solid;
  d.tau_one = h->tau_one;
  d.moving = h->p.u_wall[0] != 0.0 || h->p.u_wall[1] != 0.0;
  d.link = h->link;
  d.solid = h->solid;
  d.t_bottom = h->t_bottom;
  d.partials = partials ? partials : h->partials;
  d.fields = fields ? fields : h->fields;
  return d;
}

void launch_pass(const tlb_handle* h, tlbh::Pass pass, const void* src, void* dst,
                 double* fields = nullptr, double* partials = nullptr, void* moments = nullptr) {
  const tlbh::Device d = device_view(h, fields, partials);
  with_storage(h->p.precision,
               [&](auto st) { tlbh::Launcher<decltype(st)>::step(d, pass, src, dst, moments); });
}

// Re-run the step that produced f*(t) without storing, to evaluate the
// moments, forces and u^H of time t (observables or fields).
enum class Level { kObserve, kFields, kStress };

int evaluate_time_level(tlb_handle* h, Level what, double* fields = nullptr) {
  const void* src = h->buf[1 - h->cur];
  using tlbh::Pass;
  const bool init = h->t == 0;
  Pass pass = init ? Pass::kObserveInit : Pass::kObserve;
  if (what == Level::kFields) pass = init ? Pass::kFieldsInit : Pass::kFields;
  if (what == Level::kStress) pass = init ? Pass::kStressInit : Pass::kStress;
  launch_pass(h, pass, src, nullptr, fields);
  TLB_HIP(h, hipGetLastError());
  return TLB_OK;
}

bool finite_positive(double v) { return std::isfinite(v) && v > 0; }

// Fluid-node sum of the central differences (T(y+1) - T(y-1)) / 2 with the
// mirror value 2 T_w - T(y) at a solid neighbour (Nu, Eq. (24)): along a
// column each run of fluid nodes from row a to row b telescopes to
// T_w(above b) - T_w(below a), whatever the fluid temperatures are.
double dtdy_sum(const tlb_handle* h) {
  const int lx = h->p.lx, ly = h->p.ly;
  auto wall_t = [&](int x, int y) {
    if (y < 0) return h->host_tb[x];
    if (y >= ly) return h->p.t_top;
    return h->host_solid[(size_t)y * lx + x] == 1 ? h->host_tb[x] : h->p.t_top;
  };
  double sum = 0;
  for (int x = 0; x < lx; ++x) {
    int y = 0;
    while (y < ly) {
      if (h->host_solid[(size_t)y * lx + x] != 0) {
        ++y;
        continue;
      }
      const int a = y;
      while (y < ly && h->host_solid[(size_t)y * lx + x] == 0) ++y;
      sum += wall_t(x, y) - wall_t(x, a - 1);
    }
  }
  return sum;
}

size_t state_bytes(const tlb_handle* h) {
  return buffer_planes(h->p.precision) * h->pop_stride * h->elem;
}

// Bytes of one moment-tape slot: rho_A, rho_B, j_x, j_y, T of every node in
// the compute type (the adjoint's storages: FP64, FP32).
size_t moment_bytes(const tlb_handle* h) {
  return (size_t)5 * h->pop_stride * (h->p.precision == TLB_FP64 ? sizeof(double) : sizeof(float));
}

// Device buffer of at least `bytes`, reallocated when too small.
int ensure_buffer(tlb_handle* h, void** ptr, size_t* cap, size_t bytes, const char* what) {
  if (*cap >= bytes && *ptr) return TLB_OK;
  if (*ptr) {
    TLB_HIP(h, hipStreamSynchronize(h->stream));
    TLB_HIP(h, hipFree(*ptr));
    *ptr = nullptr;
    *cap = 0;
  }
  const hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(h, e == hipErrorOutOfMemory ? TLB_ENOMEM : TLB_EDEVICE,
                "%s: hipMalloc of %zu bytes failed: %s", what, bytes, hipGetErrorString(e));
  }
  *cap = bytes;
  return TLB_OK;
}

// Slots per step of the taped run's loss terms: one per strip of the fused
// kernel (whose launches write per-strip top-row sums), else one.
int loss_stride(const tlb_handle* h) {
  return h->launch.rows2 > 0 ? (int)h->launch.grid2.x : 1;
}

// Adjoint work buffers (planes and FP64 scalars) for a run of `nsteps`.
int ensure_adjoint_work(tlb_handle* h, int64_t nsteps, tlbh::AdjointWork* w) {
  const size_t csize = is_fp64(h) ? sizeof(double) : sizeof(float);
  const size_t plane = (size_t)h->pop_stride * csize;
  size_t cap = h->adj ? (size_t)tlbh::kAdjointPlanes * plane : 0;
  int rc = ensure_buffer(h, &h->adj, &cap, (size_t)tlbh::kAdjointPlanes * plane, "adjoint work");
  if (rc != TLB_OK) return rc;
  const size_t scalars = (size_t)h->p.lx + (size_t)nsteps * (size_t)loss_stride(h);
  size_t scap = h->adj_scalars ? ((size_t)h->p.lx + h->loss_cap) * sizeof(double) : 0;
  rc = ensure_buffer(h, reinterpret_cast<void**>(&h->adj_scalars), &scap, scalars * sizeof(double),
                     "adjoint scalars");
  if (rc != TLB_OK) return rc;
  h->loss_cap = scap / sizeof(double) - (size_t)h->p.lx;
  char* base = static_cast<char*>(h->adj);
  w->lam[0] = base;
  w->lam[1] = base + 27 * plane;
  w->fbar = base + 54 * plane;
  w->Fbar = base + 81 * plane;
  w->aux = base + 85 * plane;
  w->rbar = base + 89 * plane;
  w->grad = h->adj_scalars;
  w->loss_terms = h->adj_scalars + h->p.lx;
  return TLB_OK;
}

// Call f with the storage policy of an FP64 / FP32 handle.
template <class F>
void with_adjoint_storage(const tlb_handle* h, F&& f) {
  if (is_fp64(h)) f(tlbk::Store<double>{});
  else f(tlbk::Store<float>{});
}

// Device buffers of one droplet detection: the fields of the time level
// ([5][ly][lx]), per node parent / root number / label ([3][ly*lx]), the
// per-tile root counts and their offsets, the error flag, the FP64 bottom
// temperature ([lx]) and per droplet 7 int64 sums, the root and the output
// record (`acc`, room for `acc_count` droplets).
struct DropBuffers {
  double* fields = nullptr;
  int32_t* nodes = nullptr;
  int32_t* tiles = nullptr;
  int* error = nullptr;
  double* tb = nullptr;
  void* acc = nullptr;
  int64_t acc_count = 0;
};

constexpr size_t kDropBytesPerDroplet =
    7 * sizeof(int64_t) + sizeof(int64_t) + sizeof(tlbk::DropRecord);
static_assert(sizeof(tlbk::DropRecord) == sizeof(tlb_droplet), "droplet record layout");
static_assert(offsetof(tlb_droplet, nu) == offsetof(tlbk::DropRecord, nu), "droplet record layout");

// Static workspace of tlb_droplets_noalloc: one array per device, sized for
// lattices of up to kNoAllocNodes nodes and kNoAllocCols columns with up to
// kNoAllocDroplets droplets. Layout (each part 256-byte aligned): fields
// [5][n] doubles, nodes [3][n] int32, tile counts, error flag, FP64 bottom
// temperature [lx], per-droplet accumulators.
constexpr int64_t kNoAllocNodes = int64_t(1) << 19;
constexpr int64_t kNoAllocCols = 8192;
constexpr int64_t kNoAllocDroplets = int64_t(1) << 14;
constexpr size_t align256(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t kNoAllocTiles = (kNoAllocNodes + tlbk::kDropTile - 1) / tlbk::kDropTile + 1;
constexpr size_t kNoAllocOffNodes = align256(5 * kNoAllocNodes * sizeof(double));
constexpr size_t kNoAllocOffTiles = kNoAllocOffNodes + align256(3 * kNoAllocNodes * sizeof(int32_t));
constexpr size_t kNoAllocOffError = kNoAllocOffTiles + align256(kNoAllocTiles * sizeof(int32_t));
constexpr size_t kNoAllocOffTb = kNoAllocOffError + 256;
constexpr size_t kNoAllocOffAcc = kNoAllocOffTb + align256(kNoAllocCols * sizeof(double));
constexpr size_t kNoAllocBytes = kNoAllocOffAcc + align256(kNoAllocDroplets * kDropBytesPerDroplet);

}  // namespace

// In host code `scratch` names a host-side stand-in; the device address of
// each GPU's copy comes from hipGetSymbolAddress (scratch_address).
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), looked up
// once per device; nullptr with the HIP error in *err on failure.
void* scratch_address(int device, hipError_t* err) {
  *err = hipSuccess;
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

// Droplet detection into `b`. `grow` reallocates the per-droplet buffer of
// the handle when the count exceeds it; without it more droplets than
// b.acc_count is an error.
int run_droplets(tlb_handle* h, const char* who, DropBuffers& b, bool grow, double threshold,
                 tlb_droplet* out, int64_t cap, int64_t* count, int32_t* labels) {
  const int lx = h->p.lx, ly = h->p.ly;
  const int n = lx * ly;  // below 2^30 (checked at init)
  const int tiles = (n + tlbk::kDropTile - 1) / tlbk::kDropTile;
  int rc = evaluate_time_level(h, Level::kFields, b.fields);
  if (rc != TLB_OK) return rc;
  hipLaunchKernelGGL(tlbk::drop_bottom_temperature, dim3((lx + 255) / 256), dim3(256), 0,
                     h->stream, h->t_bottom, is_fp64(h) ? 0 : 1, b.tb, lx, b.error);
  tlbk::DropArgs a{};
  a.fields = b.fields;
  a.solid = h->solid;
  a.t_bottom = b.tb;
  a.parent = b.nodes;
  a.rid = b.nodes + n;
  a.label = b.nodes + 2 * (size_t)n;
  a.block_count = b.tiles;
  a.error = b.error;
  a.threshold = threshold;
  a.t_top = h->p.t_top;
  a.kappa = (h->p.tau_g - 0.5) / 3.0;
  a.dt_nominal = h->p.dt_nominal;
  a.lx = lx;
  a.ly = ly;
  a.n = n;
  const dim3 block(256);
  const dim3 local_tiles((lx + tlbk::kLocalW - 1) / tlbk::kLocalW,
                         (ly + tlbk::kLocalH - 1) / tlbk::kLocalH);
  const dim3 acc_tiles((lx + tlbk::kLocalW - 1) / tlbk::kLocalW,
                       (ly + tlbk::kAccRows - 1) / tlbk::kAccRows);
  hipLaunchKernelGGL(tlbk::drop_local, local_tiles, block, 0, h->stream, a);
  const dim3 borders((unsigned)((tlbk::border_links(lx, ly) + 255) / 256));
  if (borders.x > 0) hipLaunchKernelGGL(tlbk::drop_union_border, borders, block, 0, h->stream, a);
  hipLaunchKernelGGL(tlbk::drop_count_roots, dim3(tiles), block, 0, h->stream, a);
  hipLaunchKernelGGL(tlbk::drop_scan_tiles, dim3(1), block, 0, h->stream, b.tiles, tiles);
  a.total = b.tiles + tiles;
  // Numbering, sums and records for the droplets the buffer has room for,
  // launched without waiting for the count (kernels read it on the device);
  // when the count exceeds the room, a growing call repeats this part.
  auto sums = [&]() {
    a.acc = static_cast<int64_t*>(b.acc);
    a.roots = a.acc + 7 * (size_t)b.acc_count;
    a.out = reinterpret_cast<tlbk::DropRecord*>(a.roots + b.acc_count);
    a.capacity = (int)b.acc_count;
    const dim3 per_droplet((unsigned)((b.acc_count + 255) / 256));
    if (b.acc_count > 0)
      hipLaunchKernelGGL(tlbk::drop_clear, per_droplet, block, 0, h->stream, a.acc, a.total,
                         a.capacity);
    hipLaunchKernelGGL(tlbk::drop_number_roots, dim3(tiles), block, 0, h->stream, a);
    hipLaunchKernelGGL(tlbk::drop_accumulate, acc_tiles, block, 0, h->stream, a);
    if (b.acc_count > 0)
      hipLaunchKernelGGL(tlbk::drop_finalize, per_droplet, block, 0, h->stream, a);
  };
  sums();
  TLB_HIP(h, hipGetLastError());
  int32_t total = 0;
  int err = 0;
  TLB_HIP(h, hipMemcpyAsync(&total, a.total, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  TLB_HIP(h, hipMemcpyAsync(&err, b.error, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  TLB_HIP(h, hipStreamSynchronize(h->stream));
  if (err) return fail(h, TLB_EDEVICE, "%s: cluster walk exceeded its bound", who);
  *count = total;
  if (total > b.acc_count) {
    if (!grow)
      return fail(h, TLB_EINVAL, "%s: %d droplets, more than the workspace holds (%lld)", who,
                  (int)total, (long long)b.acc_count);
    if (h->drop_acc) TLB_HIP(h, hipFree(h->drop_acc));
    h->drop_acc = nullptr;
    h->drop_acc_cap = 0;
    TLB_HIP(h, hipMalloc(&h->drop_acc, (size_t)total * kDropBytesPerDroplet));
    h->drop_acc_cap = (size_t)total;
    b.acc = h->drop_acc;
    b.acc_count = total;
    sums();
    TLB_HIP(h, hipGetLastError());
  }
  const int64_t m = std::min<int64_t>(cap, total);
  if (m > 0)
    TLB_HIP(h, hipMemcpyAsync(out, a.out, (size_t)m * sizeof(tlb_droplet), hipMemcpyDeviceToHost,
                              h->stream));
  if (labels)
    TLB_HIP(h, hipMemcpyAsync(labels, a.label, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost,
                              h->stream));
  TLB_HIP(h, hipStreamSynchronize(h->stream));
  return TLB_OK;
}

}  // namespace

namespace {

// Parameter checks shared by tlb_init, tlb_init_external and
// tlb_workspace_bytes.
int check_params(const tlb_params* p) {
  if (p->lx < 1 || p->ly < 1 || (long long)p->lx * p->ly > (1LL << 30))
    return fail(nullptr, TLB_EINVAL, "tlb_init: bad lattice size %d x %d", p->lx, p->ly);
  if (p->precision < TLB_FP64 || p->precision > TLB_FIX16_DEV)
    return fail(nullptr, TLB_EINVAL, "tlb_init: unknown precision %d", p->precision);
  if (!std::isfinite(p->rho_ref[0]) || !std::isfinite(p->rho_ref[1]) || !std::isfinite(p->t_ref))
    return fail(nullptr, TLB_EINVAL, "tlb_init: rho_ref and t_ref must be finite");
  if (!std::isfinite(p->u_wall[0]) || !std::isfinite(p->u_wall[1]))
    return fail(nullptr, TLB_EINVAL, "tlb_init: u_wall must be finite");
  if ((p->launch_flags & ~(TLB_LAUNCH_GENERAL_PATH | TLB_LAUNCH_WIDE_OFFSETS)) != 0 ||
      p->fused < TLB_FUSED_AUTO || p->fused > TLB_FUSED_ALWAYS || p->fused_rows < 0 ||
      p->fused_rows > 4096 || p->fused_strip < 0 ||
      p->fused_strip >= tlbh::kStep2Lanes - tlbh::kStep2Halo || p->rows < 0 || p->rows > 4096 ||
      (p->fused_lanes != 0 && p->fused_lanes != tlbh::kStep2Lanes &&
       p->fused_lanes != tlbh::kStep2LanesNarrow))
    return fail(nullptr, TLB_EINVAL,
                "tlb_init: launch options out of range (flags %d, fused %d, fused_rows %d, "
                "fused_strip %d, rows %d, fused_lanes %d)",
                p->launch_flags, p->fused, p->fused_rows, p->fused_strip, p->rows, p->fused_lanes);
  if (!(p->tau > 0.5) || !(p->tau_g > 0.5) || !finite_positive(p->rho0) || !(p->dt_nominal != 0) ||
      !std::isfinite(p->dt_nominal))
    return fail(nullptr, TLB_EINVAL, "tlb_init: need tau > 1/2, tau_g > 1/2, rho0 > 0, dt_nominal != 0");
  return TLB_OK;
}

// Layout of the step path's device buffers (each part 256-byte aligned):
// both population buffers, the per-block observable partials, the
// observables, the bottom temperature, the solid flags and the link masks.
struct Workspace {
  size_t buf = 0, partials = 0, obs = 0, t_bottom = 0, solid = 0, link = 0, total = 0;
};

Workspace workspace_layout(const tlb_params& p, size_t state_b, size_t nblocks) {
  const size_t n = (size_t)p.lx * p.ly;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  Workspace w;
  w.buf = 0;
  w.partials = 2 * up(state_b);
  w.obs = w.partials + up(nblocks * tlbk::kObsSums * sizeof(double));
  w.t_bottom = w.obs + up(8 * sizeof(double));
  w.solid = w.t_bottom + up((size_t)p.lx * sizeof(double));
  w.link = w.solid + up(n);
  w.total = w.link + up(n * sizeof(uint16_t));
  return w;
}

bool any_solid(const uint8_t* solid, size_t n) {
  if (!solid) return false;
  for (size_t q = 0; q < n; ++q)
    if (solid[q] != 0) return true;
  return false;
}

int init_impl(tlb_handle** out, const tlb_params* p, const double* rho_a, const double* rho_b,
              const double* temp, const double* ux0, const double* uy0, const uint8_t* solid,
              const double* t_bottom, void* hip_stream, void* workspace, size_t workspace_bytes) {
  g_init_error[0] = 0;
  if (!out) return fail(nullptr, TLB_EINVAL, "tlb_init: out is NULL");
  *out = nullptr;
  if (!p || !rho_a || !rho_b || !temp || !t_bottom)
    return fail(nullptr, TLB_EINVAL, "tlb_init: NULL params or field array");
  int prc = check_params(p);
  if (prc != TLB_OK) return prc;
  if (workspace && (reinterpret_cast<uintptr_t>(workspace) % 256) != 0)
    return fail(nullptr, TLB_EINVAL, "tlb_init_external: workspace not 256-byte aligned");

  tlb_handle* h = new (std::nothrow) tlb_handle();
  if (!h) return fail(nullptr, TLB_ENOMEM, "tlb_init: host allocation failed");
  h->p = *p;
  const int lx = p->lx, ly = p->ly;
  const size_t n = (size_t)lx * ly;

  // host-side pre-processing: solid flags and link masks
  std::vector<uint8_t> sol(n, 0);
  if (solid) {
    for (size_t q = 0; q < n; ++q) {
      if (solid[q] > 2) {
        delete h;
        return fail(nullptr, TLB_EINVAL, "tlb_init: solid flag %d at %zu (0, 1 or 2 expected)",
                    (int)solid[q], q);
      }
      sol[q] = solid[q];
      h->has_solid |= solid[q] != 0;
    }
  }
  std::vector<uint16_t> link;
  if (h->has_solid) {
    link.assign(n, 0);
    for (int y = 0; y < ly; ++y)
      for (int x = 0; x < lx; ++x) {
        uint16_t m = sol[(size_t)y * lx + x] ? 1 : 0;
        for (int i = 1; i < 9; ++i) {
          const int sx = ((x - tlbk::dir_cx(i)) % lx + lx) % lx;
          const int sy = y - tlbk::dir_cy(i);
          const bool s = sy < 0 || sy >= ly || sol[(size_t)sy * lx + sx] != 0;
          if (s) m |= (uint16_t)(1u << i);
        }
        link[(size_t)y * lx + x] = m;
      }
  }
  for (size_t q = 0; q < n; ++q) h->n_fluid += sol[q] == 0;
  h->host_solid = sol;
  for (int x = 0; x < lx; ++x) h->n_top += sol[(size_t)(ly - 1) * lx + x] == 0;

  h->pitch = (lx + 63) / 64 * 64;
  h->pop_stride = (long long)h->pitch * ly;
  h->elem = storage_bytes(p->precision);
  // tau = tau_g = 1 gives f* = f^eq exactly: the kernels keep only moments of
  // the pulled rows (TLB_LAUNCH_GENERAL_PATH forces the general path)
  h->tau_one = p->tau == 1.0 && p->tau_g == 1.0 && !(p->launch_flags & TLB_LAUNCH_GENERAL_PATH);
  h->launch = choose_launch(*p, buffer_planes(p->precision) * h->pop_stride * h->elem,
                            h->has_solid, h->tau_one);

  int rc = TLB_OK;
  auto cleanup_fail = [&](int code) {
    tlb_destroy(h);
    return code;
  };
  if (hip_stream) {
    h->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    hipError_t e = hipStreamCreate(&h->stream);
    if (e != hipSuccess) {
      fail(nullptr, TLB_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
      delete h;
      return TLB_EDEVICE;
    }
    h->own_stream = true;
  }
  {
    // the device's copy of the no-allocation workspace (tlb_droplets_noalloc)
    hipError_t e = hipGetDevice(&h->device);
    if (e == hipSuccess) (void)scratch_address(h->device, &e);
    if (e != hipSuccess) {
      fail(nullptr, TLB_EDEVICE, "tlb_init: device workspace lookup: %s", hipGetErrorString(e));
      tlb_destroy(h);
      return TLB_EDEVICE;
    }
  }

#define INIT_HIP(expr)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      fail(nullptr, e_ == hipErrorOutOfMemory ? TLB_ENOMEM : TLB_EDEVICE, "%s: %s", #expr, \
           hipGetErrorString(e_));                                                      \
      return cleanup_fail(e_ == hipErrorOutOfMemory ? TLB_ENOMEM : TLB_EDEVICE);       \
    }                                                                                   \
  } while (0)

  const size_t buf_bytes = state_bytes(h);
  const size_t nblocks = (size_t)h->launch.grid.x * h->launch.grid.y;
  if (workspace) {
    const Workspace ws = workspace_layout(*p, buf_bytes, nblocks);
    if (workspace_bytes < ws.total) {
      fail(nullptr, TLB_EINVAL, "tlb_init_external: workspace of %zu bytes, %zu needed",
           workspace_bytes, ws.total);
      return cleanup_fail(TLB_EINVAL);
    }
    char* base = static_cast<char*>(workspace);
    h->external = true;
    h->buf[0] = base + ws.buf;
    h->buf[1] = base + ws.buf + (ws.partials - ws.buf) / 2;
    h->partials = reinterpret_cast<double*>(base + ws.partials);
    h->obs = reinterpret_cast<double*>(base + ws.obs);
    h->t_bottom = base + ws.t_bottom;
    h->solid = reinterpret_cast<uint8_t*>(base + ws.solid);
    if (h->has_solid) h->link = reinterpret_cast<uint16_t*>(base + ws.link);
  } else {
    INIT_HIP(hipMalloc(&h->buf[0], buf_bytes));
    INIT_HIP(hipMalloc(&h->buf[1], buf_bytes));
    INIT_HIP(hipMalloc(&h->partials, nblocks * tlbk::kObsSums * sizeof(double)));
    INIT_HIP(hipMalloc(&h->obs, 8 * sizeof(double)));
    INIT_HIP(hipMalloc(&h->t_bottom, lx * (is_fp64(h) ? sizeof(double) : sizeof(float))));
    INIT_HIP(hipMalloc(&h->solid, n));
    if (h->has_solid) INIT_HIP(hipMalloc(&h->link, n * sizeof(uint16_t)));
  }
  INIT_HIP(hipMemsetAsync(h->buf[1], 0, buf_bytes, h->stream));
  INIT_HIP(hipMemcpyAsync(h->solid, sol.data(), n, hipMemcpyHostToDevice, h->stream));
  if (h->has_solid)
    INIT_HIP(hipMemcpyAsync(h->link, link.data(), n * sizeof(uint16_t), hipMemcpyHostToDevice,
                            h->stream));
  rc = tlb_set_bottom_temperature(h, t_bottom);
  if (rc != TLB_OK) {
    snprintf(g_init_error, sizeof g_init_error, "%s", h->err);
    return cleanup_fail(rc);
  }

  // initial fields (staged in buf[0], which holds at least 40 bytes per
  // node) -> f(0) in buf[1] -> f*(0) in buf[0]
  double* d_fields = static_cast<double*>(h->buf[0]);
  const int nf = (ux0 && uy0) ? 5 : 3;
  const double* srcs[5] = {rho_a, rho_b, temp, ux0, uy0};
  for (int k = 0; k < nf; ++k)
    INIT_HIP(hipMemcpyAsync(d_fields + k * n, srcs[k], n * sizeof(double), hipMemcpyHostToDevice,
                            h->stream));
  const double* dux = nf == 5 ? d_fields + 3 * n : nullptr;
  const double* duy = nf == 5 ? d_fields + 4 * n : nullptr;
  {
    const tlbh::Device d = device_view(h);
    with_storage(p->precision, [&](auto st) {
      tlbh::Launcher<decltype(st)>::init_equilibrium(d, h->buf[1], d_fields, d_fields + n,
                                                     d_fields + 2 * n, dux, duy);
    });
  }
  INIT_HIP(hipGetLastError());
  INIT_HIP(hipMemsetAsync(h->buf[0], 0, buf_bytes, h->stream));
  launch_pass(h, tlbh::Pass::kInitStep, h->buf[1], h->buf[0]);
  INIT_HIP(hipGetLastError());
  h->obs_t = 0;
  INIT_HIP(hipStreamSynchronize(h->stream));
#undef INIT_HIP
  h->cur = 0;
  h->t = 0;
  *out = h;
  return TLB_OK;
}

}  // namespace

extern "C" {

int tlb_init(tlb_handle** out, const tlb_params* p, const double* rho_a, const double* rho_b,
             const double* temp, const double* ux0, const double* uy0, const uint8_t* solid,
             const double* t_bottom, void* hip_stream) {
  return init_impl(out, p, rho_a, rho_b, temp, ux0, uy0, solid, t_bottom, hip_stream, nullptr, 0);
}

int tlb_init_external(tlb_handle** out, const tlb_params* p, const double* rho_a,
                      const double* rho_b, const double* temp, const double* ux0,
                      const double* uy0, const uint8_t* solid, const double* t_bottom,
                      void* hip_stream, void* workspace, int64_t workspace_bytes) {
  if (!workspace || workspace_bytes <= 0) {
    g_init_error[0] = 0;
    if (out) *out = nullptr;
    return fail(nullptr, TLB_EINVAL, "tlb_init_external: NULL or empty workspace");
  }
  return init_impl(out, p, rho_a, rho_b, temp, ux0, uy0, solid, t_bottom, hip_stream, workspace,
                   (size_t)workspace_bytes);
}

int64_t tlb_workspace_bytes(const tlb_params* p, const uint8_t* solid) {
  if (!p) return fail(nullptr, TLB_EINVAL, "tlb_workspace_bytes: NULL params");
  int rc = check_params(p);
  if (rc != TLB_OK) return rc;
  const size_t n = (size_t)p->lx * p->ly;
  const bool has_solid = any_solid(solid, n);
  const long long pitch = (p->lx + 63) / 64 * 64;
  const size_t state_b = buffer_planes(p->precision) * (size_t)(pitch * p->ly) *
                         storage_bytes(p->precision);
  const bool tau_one = p->tau == 1.0 && p->tau_g == 1.0 && !(p->launch_flags & TLB_LAUNCH_GENERAL_PATH);
  const tlbh::Geometry g = choose_launch(*p, state_b, has_solid, tau_one);
  return (int64_t)workspace_layout(*p, state_b, (size_t)g.grid.x * g.grid.y).total;
}

int tlb_step(tlb_handle* h, int64_t nsteps) {
  if (!h) return fail(nullptr, TLB_EINVAL, "tlb_step: NULL handle");
  if (nsteps < 0) return fail(h, TLB_EINVAL, "tlb_step: nsteps < 0");
  // Fused two-step launches first; the call always ends with a single step,
  // so the other buffer holds f*(t-1), from which fields and stress of
  // time t are pulled. That last step also leaves the observable sums of
  // the new time in the partials.
  int64_t s = 0;
  if (h->launch.rows2 > 0) {
    for (; s + 2 < nsteps; s += 2) {
      launch_pass(h, tlbh::Pass::kStep2, h->buf[h->cur], h->buf[1 - h->cur]);
      h->cur = 1 - h->cur;
      h->t += 2;
    }
  }
  for (; s < nsteps; ++s) {
    const bool last = s + 1 == nsteps;
    launch_pass(h, last ? tlbh::Pass::kStepObserve : tlbh::Pass::kStep, h->buf[h->cur],
                h->buf[1 - h->cur]);
    h->cur = 1 - h->cur;
    h->t += 1;
    if (last) h->obs_t = h->t;
  }
  TLB_HIP(h, hipGetLastError());
  return TLB_OK;
}

int tlb_launch_info(const tlb_handle* h, tlb_launch* out) {
  if (!h || !out) return TLB_EINVAL;
  const tlbh::Geometry& g = h->launch;
  out->bx = g.bx;
  out->rows = g.rows;
  out->grid_x = (int32_t)g.grid.x;
  out->grid_y = (int32_t)g.grid.y;
  out->fused_rows = g.rows2;
  out->fused_strip = g.strip2;
  out->fused_grid_x = g.rows2 > 0 ? (int32_t)g.grid2.x : 0;
  out->fused_grid_y = g.rows2 > 0 ? (int32_t)g.grid2.y : 0;
  out->fused_lanes = g.rows2 > 0 ? g.lanes2 : 0;
  return TLB_OK;
}

int tlb_observables(tlb_handle* h, tlb_obs* out) {
  if (!h || !out) return fail(h, TLB_EINVAL, "tlb_observables: NULL argument");
  // the last step of tlb_step left the sums of the current time; otherwise
  // (a taped run, a new bottom temperature) re-evaluate the time level
  if (h->obs_t != h->t) {
    int rc = evaluate_time_level(h, Level::kObserve);
    if (rc != TLB_OK) return rc;
    h->obs_t = h->t;
  }
  tlbk::ObsArgs oa{};
  oa.partials = h->partials;
  oa.nblocks = (int)(h->launch.grid.x * h->launch.grid.y);
  oa.n_fluid = h->n_fluid;
  oa.n_top = h->n_top;
  oa.kappa = (h->p.tau_g - 0.5) / 3.0;
  oa.dt_nominal = h->p.dt_nominal;
  oa.ly = h->p.ly;
  oa.dtdy_sum = h->dtdy_sum;
  oa.out = h->obs;
  hipLaunchKernelGGL(tlbk::lb_reduce_observables, dim3(1), dim3(256), 0, h->stream, oa);
  TLB_HIP(h, hipGetLastError());
  double v[6];
  TLB_HIP(h, hipMemcpyAsync(v, h->obs, sizeof v, hipMemcpyDeviceToHost, h->stream));
  TLB_HIP(h, hipStreamSynchronize(h->stream));
  out->step = h->t;
  out->mass_a = v[0];
  out->mass_b = v[1];
  out->sum_t = v[2];
  out->nu = v[3];
  out->nu_top = v[4];
  out->ke = v[5];
  if (!std::isfinite(v[0]) || !std::isfinite(v[1]))
    return fail(h, TLB_ENUMERIC, "tlb_observables: non-finite mass at step %lld", (long long)h->t);
  return TLB_OK;
}

int tlb_get_fields(tlb_handle* h, double* rho_a, double* rho_b, double* ux, double* uy,
                   double* temp) {
  if (!h) return fail(nullptr, TLB_EINVAL, "tlb_get_fields: NULL handle");
  const size_t n = (size_t)h->p.lx * h->p.ly;
  if (!h->fields) TLB_HIP(h, hipMalloc(&h->fields, 7 * n * sizeof(double)));
  int rc = evaluate_time_level(h, Level::kFields);
  if (rc != TLB_OK) return rc;
  double* outs[5] = {rho_a, rho_b, ux, uy, temp};
  for (int k = 0; k < 5; ++k)
    if (outs[k])
      TLB_HIP(h, hipMemcpyAsync(outs[k], h->fields + k * n, n * sizeof(double),
                                hipMemcpyDeviceToHost, h->stream));
  TLB_HIP(h, hipStreamSynchronize(h->stream));
  return TLB_OK;
}

int tlb_get_stress(tlb_handle* h, double* sxy_visc, double* pxy_int) {
  if (!h) return fail(nullptr, TLB_EINVAL, "tlb_get_stress: NULL handle");
  const size_t n = (size_t)h->p.lx * h->p.ly;
  if (!h->fields) TLB_HIP(h, hipMalloc(&h->fields, 7 * n * sizeof(double)));
  int rc = evaluate_time_level(h, Level::kStress);
  if (rc != TLB_OK) return rc;
  double* outs[2] = {sxy_visc, pxy_int};
  for (int k = 0; k < 2; ++k)
    if (outs[k])
      TLB_HIP(h, hipMemcpyAsync(outs[k], h->fields + (5 + k) * n, n * sizeof(double),
                                hipMemcpyDeviceToHost, h->stream));
  TLB_HIP(h, hipStreamSynchronize(h->stream));
  return TLB_OK;
}

int tlb_row_averages(tlb_handle* h, double* u_av, double* pxy_av) {
  if (!h) return fail(nullptr, TLB_EINVAL, "tlb_row_averages: NULL handle");
  const int lx = h->p.lx, ly = h->p.ly;
  const size_t n = (size_t)lx * ly;
  if (!h->fields) TLB_HIP(h, hipMalloc(&h->fields, 7 * n * sizeof(double)));
  if (!h->rows) TLB_HIP(h, hipMalloc(&h->rows, 2 * (size_t)ly * sizeof(double)));
  int rc = evaluate_time_level(h, Level::kStress);
  if (rc != TLB_OK) return rc;
  hipLaunchKernelGGL(tlbk::lb_row_averages, dim3(ly), dim3(256), 0, h->stream, h->fields, h->solid,
                     lx, ly, h->rows, h->rows + ly);
  TLB_HIP(h, hipGetLastError());
  double* outs[2] = {u_av, pxy_av};
  for (int k = 0; k < 2; ++k)
    if (outs[k])
      TLB_HIP(h, hipMemcpyAsync(outs[k], h->rows + (size_t)k * ly, ly * sizeof(double),
                                hipMemcpyDeviceToHost, h->stream));
  TLB_HIP(h, hipStreamSynchronize(h->stream));
  return TLB_OK;
}

int tlb_droplets(tlb_handle* h, double threshold, tlb_droplet* out, int64_t cap, int64_t* count,
                 int32_t* labels) {
  if (!h || !count) return fail(h, TLB_EINVAL, "tlb_droplets: NULL handle or count");
  if (cap < 0 || (cap > 0 && !out))
    return fail(h, TLB_EINVAL, "tlb_droplets: need cap >= 0 and an output array when cap > 0");
  if (!std::isfinite(threshold)) return fail(h, TLB_EINVAL, "tlb_droplets: threshold not finite");
  const int lx = h->p.lx, ly = h->p.ly;
  const int n = lx * ly;
  const int tiles = (n + tlbk::kDropTile - 1) / tlbk::kDropTile;
  if (!h->fields) TLB_HIP(h, hipMalloc(&h->fields, 7 * (size_t)n * sizeof(double)));
  if (!h->drop_nodes) TLB_HIP(h, hipMalloc(&h->drop_nodes, 3 * (size_t)n * sizeof(int32_t)));
  if (!h->drop_tiles) TLB_HIP(h, hipMalloc(&h->drop_tiles, (size_t)(tiles + 1) * sizeof(int32_t)));
  if (!h->drop_error) TLB_HIP(h, hipMalloc(&h->drop_error, sizeof(int)));
  if (!h->drop_tb) TLB_HIP(h, hipMalloc(&h->drop_tb, (size_t)lx * sizeof(double)));
  DropBuffers b;
  b.fields = h->fields;
  b.nodes = h->drop_nodes;
  b.tiles = h->drop_tiles;
  b.error = h->drop_error;
  b.tb = h->drop_tb;
  if (!h->drop_acc) {
    // room for one droplet per 64 nodes at first; grown when exceeded
    const size_t room = std::max<size_t>(4096, (size_t)n / 64);
    TLB_HIP(h, hipMalloc(&h->drop_acc, room * kDropBytesPerDroplet));
    h->drop_acc_cap = room;
  }
  b.acc = h->drop_acc;
  b.acc_count = (int64_t)h->drop_acc_cap;
  return run_droplets(h, "tlb_droplets", b, true, threshold, out, cap, count, labels);
}

int tlb_droplets_noalloc(tlb_handle* h, double threshold, tlb_droplet* out, int64_t cap,
                         int64_t* count, int32_t* labels) {
  if (!h || !count) return fail(h, TLB_EINVAL, "tlb_droplets_noalloc: NULL handle or count");
  if (cap < 0 || (cap > 0 && !out))
    return fail(h, TLB_EINVAL, "tlb_droplets_noalloc: need cap >= 0 and an output array when cap > 0");
  if (!std::isfinite(threshold))
    return fail(h, TLB_EINVAL, "tlb_droplets_noalloc: threshold not finite");
  const int lx = h->p.lx, ly = h->p.ly;
  const int64_t n = (int64_t)lx * ly;
  if (n > kNoAllocNodes || lx > kNoAllocCols)
    return fail(h, TLB_EINVAL,
                "tlb_droplets_noalloc: lattice %d x %d exceeds the static workspace (at most "
                "%lld nodes and %lld columns)",
                lx, ly, (long long)kNoAllocNodes, (long long)kNoAllocCols);
  hipError_t e = hipSuccess;
  char* base = static_cast<char*>(scratch_address(h->device, &e));
  if (!base)
    return fail(h, TLB_EDEVICE, "tlb_droplets_noalloc: workspace address: %s", hipGetErrorString(e));
  DropBuffers b;
  b.fields = reinterpret_cast<double*>(base);
  b.nodes = reinterpret_cast<int32_t*>(base + kNoAllocOffNodes);
  b.tiles = reinterpret_cast<int32_t*>(base + kNoAllocOffTiles);
  b.error = reinterpret_cast<int*>(base + kNoAllocOffError);
  b.tb = reinterpret_cast<double*>(base + kNoAllocOffTb);
  b.acc = base + kNoAllocOffAcc;
  b.acc_count = kNoAllocDroplets;
  return run_droplets(h, "tlb_droplets_noalloc", b, false, threshold, out, cap, count, labels);
}

int tlb_get_populations(tlb_handle* h, double* out) {
  if (!h || !out) return fail(h, TLB_EINVAL, "tlb_get_populations: NULL argument");
  const int lx = h->p.lx, ly = h->p.ly;
  const size_t total = (size_t)27 * lx * ly;
  if (!h->export_buf) TLB_HIP(h, hipMalloc(&h->export_buf, total * sizeof(double)));
  {
    const tlbh::Device d = device_view(h);
    with_storage(h->p.precision, [&](auto st) {
      tlbh::Launcher<decltype(st)>::export_populations(d, h->buf[h->cur], h->export_buf);
    });
  }
  TLB_HIP(h, hipGetLastError());
  TLB_HIP(h, hipMemcpyAsync(out, h->export_buf, total * sizeof(double), hipMemcpyDeviceToHost,
                            h->stream));
  TLB_HIP(h, hipStreamSynchronize(h->stream));
  return TLB_OK;
}

int tlb_set_bottom_temperature(tlb_handle* h, const double* t_bottom) {
  if (!h || !t_bottom) return fail(h, TLB_EINVAL, "tlb_set_bottom_temperature: NULL argument");
  const int lx = h->p.lx;
  h->tape_valid = false;
  h->obs_t = -1;
  h->host_tb.assign(t_bottom, t_bottom + lx);
  h->dtdy_sum = dtdy_sum(h);
  if (is_fp64(h)) {
    TLB_HIP(h, hipMemcpyAsync(h->t_bottom, t_bottom, lx * sizeof(double), hipMemcpyHostToDevice,
                              h->stream));
    TLB_HIP(h, hipStreamSynchronize(h->stream));
  } else {
    std::vector<float> tb(t_bottom, t_bottom + lx);
    TLB_HIP(h, hipMemcpyAsync(h->t_bottom, tb.data(), lx * sizeof(float), hipMemcpyHostToDevice,
                              h->stream));
    TLB_HIP(h, hipStreamSynchronize(h->stream));
  }
  return TLB_OK;
}

int tlb_forward_taped(tlb_handle* h, int64_t nsteps, int32_t ckpt_every, double* loss) {
  if (!h) return fail(nullptr, TLB_EINVAL, "tlb_forward_taped: NULL handle");
  if (nsteps < 1 || ckpt_every < 0)
    return fail(h, TLB_EINVAL, "tlb_forward_taped: need nsteps >= 1 and ckpt_every >= 0");
  if (h->has_solid)
    return fail(h, TLB_EINVAL, "tlb_forward_taped: the adjoint supports flat walls only");
  if (h->p.precision != TLB_FP64 && h->p.precision != TLB_FP32)
    return fail(h, TLB_EINVAL, "tlb_forward_taped: the adjoint needs FP64 or FP32 storage");
  if (h->launch.wide)
    return fail(h, TLB_EINVAL, "tlb_forward_taped: state buffer of 4 GiB or more");
  if (h->p.u_wall[0] != 0.0 || h->p.u_wall[1] != 0.0)
    return fail(h, TLB_EINVAL, "tlb_forward_taped: the adjoint needs walls at rest");
  if (h->p.ly > 65535)
    return fail(h, TLB_EINVAL, "tlb_forward_taped: ly > 65535 rows");
  // the adjoint kernels fold x offsets of up to 2 columns by one period
  if (h->p.lx < 3) return fail(h, TLB_EINVAL, "tlb_forward_taped: lx < 3 columns");
  h->tape_valid = false;
  const size_t sb = state_bytes(h);
  if (ckpt_every == 0) {
    // every step when its tape (moments at tau = 1, else states) fits in half
    // of the free device memory; else the shortest checkpoint interval whose
    // checkpoints do
    size_t free_b = 0, total_b = 0;
    TLB_HIP(h, hipMemGetInfo(&free_b, &total_b));
    const double budget = 0.5 * (double)free_b;
    const double per_step = h->tau_one ? (double)moment_bytes(h) : (double)sb;
    if ((double)nsteps * per_step <= budget) {
      ckpt_every = 1;
    } else {
      const double k = std::ceil((double)nsteps * (double)sb / budget);
      ckpt_every = (int32_t)std::min<double>(std::max(2.0, k), (double)std::max<int64_t>(nsteps, 2));
    }
  }
  // At tau = tau_g = 1 the reverse sweep needs only the moments of each
  // step's pulled state: with ckpt_every = 1 the steps write those (5 values
  // per node) and no state is kept; otherwise states are checkpointed every
  // ckpt_every steps and each segment's moments recomputed in the sweep.
  const bool moment_tape = h->tau_one && ckpt_every == 1;
  const int64_t nck = moment_tape ? 0 : (nsteps + ckpt_every - 1) / ckpt_every;
  int rc = nck > 0 ? ensure_buffer(h, &h->ckpt, &h->ckpt_cap, (size_t)nck * sb, "checkpoints")
                   : TLB_OK;
  if (rc == TLB_OK && moment_tape)
    rc = ensure_buffer(h, &h->mtape, &h->mtape_cap, (size_t)nsteps * moment_bytes(h),
                       "moment tape");
  if (rc != TLB_OK) return rc;
  tlbh::AdjointWork w;
  rc = ensure_adjoint_work(h, nsteps, &w);
  if (rc != TLB_OK) return rc;
  const tlbh::Device d = device_view(h);
  // Pairs of steps run as one fused launch (which also writes both steps'
  // top-row sums, per strip) where the kernel applies and the state between
  // them is not a checkpoint; the other steps, and always the last one (so
  // that the other buffer holds the previous state, as after tlb_step), are
  // single steps with the top-row sum of their pulled state.
  const int stride = loss_stride(h);
  const bool fused = h->launch.rows2 > 0;
  auto top_row = [&](const void* state, int64_t k) {
    with_adjoint_storage(h, [&](auto st) {
      tlbh::Adjoint<decltype(st)>::top_row_term(d, w, state, (int)k, stride);
    });
  };
  auto advance = [&](int n) {
    h->cur = 1 - h->cur;
    h->t += n;
  };
  if (moment_tape) {
    auto mslot = [&](int64_t k) { return static_cast<char*>(h->mtape) + (size_t)k * moment_bytes(h); };
    int64_t k = 0;
    for (; fused && k + 2 < nsteps; k += 2) {
      launch_pass(h, tlbh::Pass::kStep2MomentsTopRow, h->buf[h->cur], h->buf[1 - h->cur], nullptr,
                  w.loss_terms + (size_t)k * stride, mslot(k));
      advance(2);
    }
    for (; k < nsteps; ++k) {
      top_row(h->buf[h->cur], k);
      launch_pass(h, tlbh::Pass::kStepMoments, h->buf[h->cur], h->buf[1 - h->cur], nullptr,
                  nullptr, mslot(k));
      advance(1);
    }
  } else if (ckpt_every == 1) {
    // tau != 1, every state kept: the steps write each state f*(t0 + k),
    // k < nsteps, straight into its slot, so the sweep recomputes nothing;
    // the last step runs from the handle's buffer, which then holds f*(t-1)
    // as after tlb_step
    auto slot = [&](int64_t k) { return static_cast<char*>(h->ckpt) + (size_t)k * sb; };
    TLB_HIP(h, hipMemcpyAsync(slot(0), h->buf[h->cur], sb, hipMemcpyDeviceToDevice, h->stream));
    for (int64_t k = 0; k + 1 < nsteps; ++k) {
      top_row(slot(k), k);
      launch_pass(h, tlbh::Pass::kStep, slot(k), slot(k + 1));
    }
    TLB_HIP(h, hipMemcpyAsync(h->buf[h->cur], slot(nsteps - 1), sb, hipMemcpyDeviceToDevice,
                              h->stream));
    top_row(h->buf[h->cur], nsteps - 1);
    launch_pass(h, tlbh::Pass::kStep, h->buf[h->cur], h->buf[1 - h->cur]);
    h->cur = 1 - h->cur;
    h->t += nsteps;
  }
  for (int64_t k = 0; ckpt_every > 1 && k < nsteps;) {
    if (k % ckpt_every == 0)
      TLB_HIP(h, hipMemcpyAsync(static_cast<char*>(h->ckpt) + (size_t)(k / ckpt_every) * sb,
                                h->buf[h->cur], sb, hipMemcpyDeviceToDevice, h->stream));
    if (fused && k + 2 < nsteps && (k + 1) % ckpt_every != 0) {
      launch_pass(h, tlbh::Pass::kStep2TopRow, h->buf[h->cur], h->buf[1 - h->cur], nullptr,
                  w.loss_terms + (size_t)k * stride);
      advance(2);
      k += 2;
      continue;
    }
    top_row(h->buf[h->cur], k);
    launch_pass(h, tlbh::Pass::kStep, h->buf[h->cur], h->buf[1 - h->cur]);
    advance(1);
    k += 1;
  }
  TLB_HIP(h, hipGetLastError());
  std::vector<double> terms((size_t)nsteps * stride);
  TLB_HIP(h, hipMemcpyAsync(terms.data(), w.loss_terms, terms.size() * sizeof(double),
                            hipMemcpyDeviceToHost, h->stream));
  TLB_HIP(h, hipStreamSynchronize(h->stream));
  double acc = 0;   // fixed order: step by step, strip by strip
  for (double v : terms) acc += v;
  if (loss)
    *loss = acc * 2.0 * h->p.ly / (h->p.dt_nominal * h->p.lx) / (double)nsteps;
  h->taped_steps = nsteps;
  h->ckpt_every = ckpt_every;
  h->tape_valid = true;
  return TLB_OK;
}

int tlb_adjoint_step(tlb_handle* h, int64_t nsteps, double seed, double* grad_t_bottom) {
  if (!h) return fail(nullptr, TLB_EINVAL, "tlb_adjoint_step: NULL handle");
  if (!grad_t_bottom) return fail(h, TLB_EINVAL, "tlb_adjoint_step: NULL grad_t_bottom");
  if (!h->tape_valid) return fail(h, TLB_ESTATE, "tlb_adjoint_step: no valid tape");
  if (nsteps != h->taped_steps)
    return fail(h, TLB_ESTATE, "tlb_adjoint_step: %lld steps requested, the tape holds %lld",
                (long long)nsteps, (long long)h->taped_steps);
  const int K = h->ckpt_every;
  const size_t sb = state_bytes(h), mb = moment_bytes(h);
  // tau = 1: moments of the pulled states (all of them with K = 1; with K > 1
  // two segments' worth, recomputed through two scratch states on the side
  // stream while the main stream sweeps the segment after); else states (a
  // segment's K - 1 recomputed ones)
  const bool moments = h->tau_one;
  int rc = TLB_OK;
  if (moments && K > 1) {
    rc = ensure_buffer(h, &h->tape, &h->tape_cap, 2 * sb, "tape");
    if (rc == TLB_OK)
      rc = ensure_buffer(h, &h->mtape, &h->mtape_cap, 2 * (size_t)K * mb, "moment tape");
    if (rc == TLB_OK && !h->side) {
      TLB_HIP(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
      for (hipEvent_t& e : h->ev_side) TLB_HIP(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      for (hipEvent_t& e : h->ev_main) TLB_HIP(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
  } else if (!moments && K > 1) {
    rc = ensure_buffer(h, &h->tape, &h->tape_cap, (size_t)(K - 1) * sb, "tape");
  }
  if (rc != TLB_OK) return rc;
  tlbh::AdjointWork w;
  rc = ensure_adjoint_work(h, nsteps, &w);
  if (rc != TLB_OK) return rc;
  const size_t csize = is_fp64(h) ? sizeof(double) : sizeof(float);
  TLB_HIP(h, hipMemsetAsync(w.lam[0], 0, (size_t)27 * h->pop_stride * csize, h->stream));
  TLB_HIP(h, hipMemsetAsync(w.grad, 0, (size_t)h->p.lx * sizeof(double), h->stream));
  // dL/dT(x) of each top-row node at each step
  const double kappa_top = seed * 2.0 * h->p.ly / (h->p.dt_nominal * h->p.lx * (double)nsteps);
  const tlbh::Device d = device_view(h);
  const bool fused = h->launch.rows2 > 0;
  // segments swept in reverse; the full moment tape is one segment
  const int64_t seg_len = moments && K == 1 ? nsteps : K;
  const int64_t nseg = (nsteps + seg_len - 1) / seg_len;
  int in = 0;
  bool first = true, ready = false;
  auto reverse = [&](const void* state, const void* next) {
    with_adjoint_storage(h, [&](auto st) {
      tlbh::Adjoint<decltype(st)>::reverse_step(d, w, state, in, kappa_top, next, ready, first);
    });
    ready = next != nullptr;
    first = false;
    in = 1 - in;
  };
  // tau = 1, K > 1: the moments of segment `seg` (steps s0 .. s0 + len - 1)
  // from its checkpoint through the two scratch states, on the side stream,
  // into half seg % 2 of the moment tape
  tlbh::Device side = d;
  side.stream = h->side;
  auto mseg = [&](int64_t seg, int64_t j) {
    return static_cast<char*>(h->mtape) + ((size_t)(seg % 2) * K + (size_t)j) * mb;
  };
  auto recompute = [&](int64_t seg) {
    const int len = (int)std::min<int64_t>(K, nsteps - seg * K);
    const void* src = static_cast<char*>(h->ckpt) + (size_t)seg * sb;
    int b = 0;
    for (int j = 0; j < len;) {
      void* dst = static_cast<char*>(h->tape) + (size_t)b * sb;
      const bool pair = fused && j + 1 < len;
      with_storage(h->p.precision, [&](auto st) {
        tlbh::Launcher<decltype(st)>::step(
            side, pair ? tlbh::Pass::kStep2Moments : tlbh::Pass::kStepMoments, src, dst, mseg(seg, j));
      });
      j += pair ? 2 : 1;
      src = dst;
      b = 1 - b;
    }
  };
  if (moments && K > 1) {
    // the side stream starts after the main stream's work so far
    TLB_HIP(h, hipEventRecord(h->ev_main[2], h->stream));
    TLB_HIP(h, hipStreamWaitEvent(h->side, h->ev_main[2], 0));
    recompute(nseg - 1);
    TLB_HIP(h, hipEventRecord(h->ev_side[(nseg - 1) % 2], h->side));
  }
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int64_t s0 = seg * seg_len;
    const int len = (int)std::min<int64_t>(seg_len, nsteps - s0);
    if (moments && K > 1) {
      // recompute the segment before on the side stream once the sweep of
      // the segment after (which used the same half of the moment tape) is
      // done, then sweep this one when its own recompute is done
      if (seg > 0) {
        if (seg + 1 < nseg) TLB_HIP(h, hipStreamWaitEvent(h->side, h->ev_main[(seg + 1) % 2], 0));
        recompute(seg - 1);
        TLB_HIP(h, hipEventRecord(h->ev_side[(seg - 1) % 2], h->side));
      }
      TLB_HIP(h, hipStreamWaitEvent(h->stream, h->ev_side[seg % 2], 0));
      // the segment's first reverse step cannot prepare the next one's
      // densities: the previous segment is not recomputed yet
      ready = false;
      for (int j = len - 1; j >= 0; --j) reverse(mseg(seg, j), j > 0 ? mseg(seg, j - 1) : nullptr);
      TLB_HIP(h, hipEventRecord(h->ev_main[seg % 2], h->stream));
      continue;
    }
    if (moments) {
      auto mslot = [&](int64_t j) { return static_cast<char*>(h->mtape) + (size_t)(s0 + j) * mb; };
      for (int j = len - 1; j >= 0; --j) reverse(mslot(j), j > 0 ? mslot(j - 1) : nullptr);
      continue;
    }
    auto slot = [&](int j) -> void* {
      return j == 0 ? static_cast<char*>(h->ckpt) + (size_t)seg * sb
                    : static_cast<char*>(h->tape) + (size_t)(j - 1) * sb;
    };
    // tau != 1: recompute the segment's states with single steps
    for (int j = 1; j < len; ++j) launch_pass(h, tlbh::Pass::kStep, slot(j - 1), slot(j));
    // within a segment each reverse step also prepares the densities of the
    // next one's state (the previous slot); the segment's first step (j = 0)
    // cannot, the previous segment is not recomputed yet, except with every
    // state kept (K = 1), whose previous state is a checkpoint
    if (K > 1) ready = false;
    for (int j = len - 1; j >= 0; --j) {
      void* next = j > 0    ? slot(j - 1)
                   : K == 1 && seg > 0 ? static_cast<char*>(h->ckpt) + (size_t)(seg - 1) * sb
                                       : nullptr;
      reverse(slot(j), next);
    }
  }
  TLB_HIP(h, hipGetLastError());
  TLB_HIP(h, hipMemcpyAsync(grad_t_bottom, w.grad, (size_t)h->p.lx * sizeof(double),
                            hipMemcpyDeviceToHost, h->stream));
  TLB_HIP(h, hipStreamSynchronize(h->stream));
  return TLB_OK;
}

int64_t tlb_time(const tlb_handle* h) { return h ? h->t : -1; }

int tlb_destroy(tlb_handle* h) {
  if (!h) return TLB_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->external) {  // the caller's workspace
    h->buf[0] = h->buf[1] = h->t_bottom = nullptr;
    h->link = nullptr;
    h->solid = nullptr;
    h->partials = h->obs = nullptr;
  }
  void* ptrs[] = {h->buf[0],   h->buf[1],     h->link,       h->solid,      h->t_bottom,
                  h->partials, h->obs,        h->fields,     h->rows,       h->export_buf,
                  h->ckpt,     h->tape,       h->mtape,      h->adj,        h->adj_scalars,
                  h->drop_nodes, h->drop_tiles, h->drop_error, h->drop_tb,  h->drop_acc};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (hipEvent_t e : h->ev_side)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->ev_main)
    if (e) (void)hipEventDestroy(e);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return TLB_OK;
}

const char* tlb_last_error(const tlb_handle* h) { return h ? h->err : g_init_error; }

}  // extern "C"
