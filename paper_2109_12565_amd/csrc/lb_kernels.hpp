// Device code of the thermal two-component Shan-Chen lattice Boltzmann step
// (arXiv:2109.12565, Sec. 2) for gfx950.
//
// One fused kernel does the whole time step t -> t+1 for a strip of BX
// columns and a chunk of rows of the lattice:
//
//   pull     f(x, t+1) = f*(x - c_i, t) from the post-collision buffer
//            (Eqs. (1), (16)); a link whose source is solid is bounced back
//            (half-way, Sec. 2.2) for f and anti-bounced for g, holding the
//            wall temperature;
//   moments  rho_A, rho_B, j, T (Eqs. (4), (5), (17));
//   psi      rho/rho0 (Eq. (8)) and rho0 (1 - exp(-rho/rho0)) (Eq. (12)),
//            staged in an LDS ring of 6 rows x (BX + 4) columns: the 25-point
//            stencil of Eq. (11) needs 2 rows and 2 columns of halo;
//   forces   Eqs. (7), (10), (11) from LDS plus buoyancy (Eq. (22));
//   collide  velocity shift (Eq. (6)), u^H = u + F/(2 rho), BGK towards
//            f^eq(rho_l, u_l) (Eq. (3)) and g^eq(T, u^H) (Eq. (18));
//   store    27 aligned, coalesced stores into the other buffer.
//
// The strip marches upward one row per iteration. Iteration k pulls f_A, f_B
// at row r = y0 - 2 + k (kept in registers for two iterations), writes that
// row's densities and pseudopotentials to the ring, waits once at a barrier,
// and completes row r - 2, whose 5 x 5 neighbourhood is then in the ring.
// Rows are therefore pulled once from HBM; only the 4 halo columns per strip
// and the 4 halo rows per chunk are pulled twice. The ring has 6 slots, so a
// single barrier per row separates the writes of row r + 1 from the reads of
// row r - 2. The row loop is unrolled three times so that the three sets of
// kept populations change roles by renaming, not by register moves.
//
// Memory layout: population p (0..26) of node (x, y) lives at element
// p * pop_stride + y * pitch + x of a buffer; pitch is a multiple of 64
// elements so every wavefront row access is aligned. Addresses are formed as
// a uniform base pointer plus a 32-bit byte offset (kWide = false, buffers
// below 4 GiB), which maps to the scalar-base + vector-offset form of the
// global loads and stores; kWide = true uses 64-bit offsets.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace tlbk {

// ---------------------------------------------------------------- lattice
// D2Q9 velocities (Sec. 2.1, Fig. 1(b)) in the library's direction order.
template <int I> struct Dir;
template <> struct Dir<0> { static constexpr int cx = 0,  cy = 0,  opp = 0; };
template <> struct Dir<1> { static constexpr int cx = 1,  cy = 0,  opp = 3; };
template <> struct Dir<2> { static constexpr int cx = 0,  cy = 1,  opp = 4; };
template <> struct Dir<3> { static constexpr int cx = -1, cy = 0,  opp = 1; };
template <> struct Dir<4> { static constexpr int cx = 0,  cy = -1, opp = 2; };
template <> struct Dir<5> { static constexpr int cx = 1,  cy = 1,  opp = 7; };
template <> struct Dir<6> { static constexpr int cx = -1, cy = 1,  opp = 8; };
template <> struct Dir<7> { static constexpr int cx = -1, cy = -1, opp = 5; };
template <> struct Dir<8> { static constexpr int cx = 1,  cy = -1, opp = 6; };

__host__ __device__ constexpr int dir_cx(int i) {
  return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int dir_cy(int i) {
  return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
// D2Q9 weights as a function of |c|^2: 4/9, 1/9, 1/36.
template <typename C> __host__ __device__ constexpr C w_c2(int c2) {
  return c2 == 0 ? C(4) / C(9) : (c2 == 1 ? C(1) / C(9) : (c2 == 2 ? C(1) / C(36) : C(0)));
}
template <typename C> __host__ __device__ constexpr C w_dir(int i) {
  return w_c2<C>(dir_cx(i) * dir_cx(i) + dir_cy(i) * dir_cy(i));
}
// 25-point weights p(|c|^2) of Fig. 1(b) (NN + NNN shells).
template <typename C> __host__ __device__ constexpr C p_c2(int c2) {
  return c2 == 0 ? C(247) / C(420)
       : c2 == 1 ? C(4) / C(63)
       : c2 == 2 ? C(4) / C(135)
       : c2 == 4 ? C(1) / C(180)
       : c2 == 5 ? C(2) / C(945)
       : c2 == 8 ? C(1) / C(15120)
       : C(0);
}

// Link-mask bits: bit 0 = node itself is solid, bit i (1..8) = the source
// node x - c_i of direction i is solid (ghost wall row or solid cell).
constexpr uint32_t kSelfSolid = 1u;
// Directions whose source lies below (c_y = +1) / above (c_y = -1).
constexpr uint32_t kFromBelow = (1u << 2) | (1u << 5) | (1u << 6);
constexpr uint32_t kFromAbove = (1u << 4) | (1u << 7) | (1u << 8);

// ---------------------------------------------------------------- storage
// Storage policies: T is the stored type, C the compute type. The kernel
// works on values in stored form: the population itself (kDev = false) or
// its deviation from the reference w_i * ref (kDev = true). grid() maps a
// stored-form value onto the representable grid when the format is fixed
// point (kFix), where sums of stored values are exact. Stores are
// non-temporal: the next step reads the populations from HBM anyway.
template <typename T_> struct Store {
  using T = T_;
  using C = T_;
  static constexpr bool kDev = false;
  static constexpr bool kFix = false;
  __device__ static C load(const T* p) { return *p; }
  __device__ static void store(T* p, C v) { __builtin_nontemporal_store(v, p); }
  __device__ static C grid(C v) { return v; }
};

// 16-bit floating-point deviations, converted with round-to-nearest-even.
struct StoreF16Dev {
  using T = uint16_t;
  using C = float;
  static constexpr bool kDev = true;
  static constexpr bool kFix = false;
  __device__ static C grid(C v) { return v; }
  __device__ static C load(const T* p) { return (float)__builtin_bit_cast(_Float16, *p); }
  __device__ static void store(T* p, C v) {
    __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, (_Float16)v), p);
  }
};

struct StoreBF16Dev {
  using T = uint16_t;
  using C = float;
  static constexpr bool kDev = true;
  static constexpr bool kFix = false;
  __device__ static C grid(C v) { return v; }
  __device__ static C load(const T* p) { return __uint_as_float((uint32_t)*p << 16); }
  __device__ static void store(T* p, C v) {
    uint32_t u = __float_as_uint(v);
    const bool nan = (u & 0x7fffffffu) > 0x7f800000u;
    u += 0x7fffu + ((u >> 16) & 1u);  // round half to even on the dropped 16 bits
    __builtin_nontemporal_store((uint16_t)(nan ? (__float_as_uint(v) >> 16) | 0x40u : u >> 16), p);
  }
};

// 16-bit fixed-point deviations in units of 2^-15 (range [-1, 1)). Every
// stored-form value is a multiple of the unit, so sums of up to 2^8 of them
// are exact in FP32: the collision sets the rest population to the exact
// remainder and each component's mass is conserved exactly.
struct StoreFix16Dev {
  using T = int16_t;
  using C = float;
  static constexpr bool kDev = true;
  static constexpr bool kFix = true;
  static constexpr float kScale = 32768.0f;
  __device__ static C load(const T* p) { return (float)*p * (1.0f / kScale); }
  __device__ static C grid(C v) {
    const float q = fminf(fmaxf(rintf(v * kScale), -32768.0f), 32767.0f);
    return q * (1.0f / kScale);
  }
  __device__ static void store(T* p, C v) {
    __builtin_nontemporal_store((int16_t)(int)(v * kScale), p);  // v is on the grid
  }
};

// ---------------------------------------------------------------- arguments
template <typename C>
struct StepArgs {
  const void* src;          // post-collision populations f*(t) (or f(0))
  void* dst;                // receives f*(t+1)
  const uint16_t* link;     // [ly*lx] link masks (solid cells present only)
  const uint8_t* solid;     // [ly*lx] 0 fluid, 1 bottom-held, 2 top-held
  const C* t_bottom;        // [lx]
  double* partials;         // [gridDim.x*gridDim.y][8] observable sums
  double* fields;           // [5][ly][lx] rho_a, rho_b, ux, uy, T
  int lx, ly, pitch, rows_per_block;
  long long pop_stride;     // ly * pitch
  C inv_tau, inv_tau_g, tau, rho0, inv_rho0, g12;
  C ga0, ga1, gr0, gr1;
  C alpha_g, t_top, rho_wall0, rho_wall1;
  C ref_a, ref_b, ref_t;    // references of the 16-bit deviation storages
};

// Kernel variants.
enum : unsigned {
  kModeInit = 1u,     // read f(0) at the node itself instead of pulling
  kModeStore = 2u,    // write f*(t+1)
  kModeObserve = 4u,  // accumulate observable sums into partials
  kModeFields = 8u,   // write the fields
  kModeSolid = 16u,   // solid cells present: use the link masks
  kModeWide = 32u,    // 64-bit byte offsets (population buffer >= 4 GiB)
  kModeTauOne = 64u   // tau = tau_g = 1: the collision returns the equilibria
};

template <typename C> __device__ inline C psi_exp(C rho, C rho0, C inv_rho0) {
  // rho0 (1 - exp(-rho/rho0)) of Eq. (12), evaluated as -rho0 expm1(-rho/rho0)
  // to keep full relative precision at small rho.
  return -rho0 * expm1(-rho * inv_rho0);
}
__device__ inline float psi_exp(float rho, float rho0, float inv_rho0) {
  return -rho0 * expm1f(-rho * inv_rho0);
}

template <unsigned kMode>
using Off = std::conditional_t<(kMode & kModeWide) != 0, uint64_t, uint32_t>;

// Byte-offset addressing helpers (base pointer is uniform).
template <class St, unsigned kMode>
__device__ inline typename St::C ld(const void* base, Off<kMode> off) {
  return St::load(reinterpret_cast<const typename St::T*>(static_cast<const char*>(base) + off));
}
template <class St, unsigned kMode>
__device__ inline void st(void* base, Off<kMode> off, typename St::C v) {
  St::store(reinterpret_cast<typename St::T*>(static_cast<char*>(base) + off), v);
}

// Per-node addressing: byte offset of the node in a population plane, and
// the byte deltas to its x-1 and x+1 neighbours (periodic wrap included).
template <unsigned kMode>
struct NodeAddr {
  Off<kMode> own;
  Off<kMode> dxm, dxp;   // added modulo 2^32 / 2^64
};

template <class St, unsigned kMode>
__device__ inline NodeAddr<kMode> node_addr(int x, int r, int lx, Off<kMode> row_b) {
  using O = Off<kMode>;
  constexpr int E = sizeof(typename St::T);
  NodeAddr<kMode> n;
  n.own = (O)r * row_b + (O)x * E;
  n.dxm = (O)(x == 0 ? (lx - 1) * E : -E);
  n.dxp = (O)(x == lx - 1 ? -(lx - 1) * E : E);
  return n;
}

// Byte offset of the value pulled for direction I at a node (population
// plane `base` + I or its opposite on bounce-back).
template <int I, unsigned kMode>
__device__ inline Off<kMode> pull_off(const NodeAddr<kMode>& n, uint32_t lm, Off<kMode> plane_b,
                                      Off<kMode> row_b, Off<kMode> first_plane) {
  using O = Off<kMode>;
  if constexpr ((kMode & kModeInit) != 0) {
    return first_plane + (O)I * plane_b + n.own;
  } else {
    constexpr int cx = Dir<I>::cx, cy = Dir<I>::cy;
    O src = first_plane + (O)I * plane_b + n.own;
    if constexpr (cy > 0) src -= row_b;
    if constexpr (cy < 0) src += row_b;
    if constexpr (cx > 0) src += n.dxm;
    if constexpr (cx < 0) src += n.dxp;
    if constexpr (I == 0) {
      return src;
    } else {
      const O bb = first_plane + (O)Dir<I>::opp * plane_b + n.own;
      return ((lm >> I) & 1u) ? bb : src;
    }
  }
}

// Link mask of node (x, r), 0 <= r < ly.
template <unsigned kMode, typename C>
__device__ inline uint32_t link_mask(const StepArgs<C>& a, int x, int r) {
  if constexpr ((kMode & kModeSolid) != 0) {
    return a.link[(uint32_t)r * (uint32_t)a.lx + (uint32_t)x];
  } else {
    return (r == 0 ? kFromBelow : 0u) | (r == a.ly - 1 ? kFromAbove : 0u);
  }
}

// Wall temperature of the solid source of direction I seen from (x, r).
template <int I, unsigned kMode, typename C>
__device__ inline C source_wall_temperature(const StepArgs<C>& a, int x, int r) {
  constexpr int cx = Dir<I>::cx, cy = Dir<I>::cy;
  const int lx = a.lx;
  const int sx = cx > 0 ? (x == 0 ? lx - 1 : x - 1) : (cx < 0 ? (x == lx - 1 ? 0 : x + 1) : x);
  const int sr = r - cy;
  if (sr < 0) return a.t_bottom[sx];
  if (sr >= a.ly) return a.t_top;
  if constexpr ((kMode & kModeSolid) != 0) {
    return a.solid[(uint32_t)sr * (uint32_t)lx + (uint32_t)sx] == 1 ? a.t_bottom[sx] : a.t_top;
  }
  return a.t_top;
}

// Pull f_A (f[0..8]) and f_B (f[9..17]) at fluid node n, in stored form.
// Opposite directions have equal weights, so a bounced value keeps its
// deviation reference.
template <class St, unsigned kMode, typename C>
__device__ inline void pull_fluid(const void* src, const NodeAddr<kMode>& n, uint32_t lm,
                                  Off<kMode> plane_b, Off<kMode> row_b, C (&f)[18]) {
  const Off<kMode> plane9 = plane_b * 9;
#define TLB_PULL_F(I)                                                            \
  {                                                                              \
    const Off<kMode> o = pull_off<I, kMode>(n, lm, plane_b, row_b, Off<kMode>(0)); \
    f[I] = ld<St, kMode>(src, o);                                                \
    f[I + 9] = ld<St, kMode>(src, o + plane9);                                   \
  }
  TLB_PULL_F(0) TLB_PULL_F(1) TLB_PULL_F(2) TLB_PULL_F(3) TLB_PULL_F(4)
  TLB_PULL_F(5) TLB_PULL_F(6) TLB_PULL_F(7) TLB_PULL_F(8)
#undef TLB_PULL_F
}

// Pull g at fluid node (x, r), in stored form, with anti-bounce-back at
// solid sources: g_i = -g*_{opp i}(x) + 2 w_i T_w, i.e. in deviations from
// w_i T_ref: d_i = -d*_{opp i} + 2 w_i (T_w - T_ref).
template <class St, unsigned kMode, typename C>
__device__ inline void pull_thermal(const StepArgs<C>& a, const void* src, const NodeAddr<kMode>& n,
                                    uint32_t lm, Off<kMode> plane_b, Off<kMode> row_b, int x, int r,
                                    C (&g)[9]) {
  const Off<kMode> plane18 = plane_b * 18;
#define TLB_PULL_G(I)                                                                       \
  {                                                                                         \
    C v = ld<St, kMode>(src, pull_off<I, kMode>(n, lm, plane_b, row_b, plane18));           \
    if constexpr ((kMode & kModeInit) == 0 && I != 0) {                                     \
      if ((lm >> I) & 1u) {                                                                 \
        C tw = source_wall_temperature<I, kMode>(a, x, r);                                  \
        if constexpr (St::kDev) tw -= a.ref_t;                                              \
        v = St::grid(C(2) * w_dir<C>(I) * tw - v);                                          \
      }                                                                                     \
    }                                                                                       \
    g[I] = v;                                                                               \
  }
  TLB_PULL_G(0) TLB_PULL_G(1) TLB_PULL_G(2) TLB_PULL_G(3) TLB_PULL_G(4)
  TLB_PULL_G(5) TLB_PULL_G(6) TLB_PULL_G(7) TLB_PULL_G(8)
#undef TLB_PULL_G
}

template <typename C> __device__ inline C sum9(const C* f) {
  return ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
}

// Momentum sum_i c_i (f_A,i + f_B,i), x and y components.
template <typename C> __device__ inline C momentum_x(const C* fa, const C* fb) {
  return ((fa[1] - fa[3]) + (fa[5] - fa[7]) + (fa[8] - fa[6])) +
         ((fb[1] - fb[3]) + (fb[5] - fb[7]) + (fb[8] - fb[6]));
}
template <typename C> __device__ inline C momentum_y(const C* fa, const C* fb) {
  return ((fa[2] - fa[4]) + (fa[5] - fa[7]) + (fa[6] - fa[8])) +
         ((fb[2] - fb[4]) + (fb[5] - fb[7]) + (fb[6] - fb[8]));
}

// Wall temperature of a solid node (x, y) inside the lattice.
template <typename C>
__device__ inline C solid_temperature(const StepArgs<C>& a, int x, int y) {
  return a.solid[(uint32_t)y * (uint32_t)a.lx + (uint32_t)x] == 1 ? a.t_bottom[x] : a.t_top;
}

// Temperature of the neighbour (x, r) of a fluid node whose temperature is
// t_here, for the central difference of dT/dy: T itself if fluid, else the
// mirror value 2 T_w - t_here (wall plane half-way).
template <class St, unsigned kMode, typename C>
__device__ inline C neighbour_temperature(const StepArgs<C>& a, const void* src, int x, int r,
                                          C t_here, Off<kMode> plane_b, Off<kMode> row_b) {
  if (r < 0) return C(2) * a.t_bottom[x] - t_here;
  if (r >= a.ly) return C(2) * a.t_top - t_here;
  const uint32_t lm = link_mask<kMode>(a, x, r);
  if (lm & kSelfSolid) return C(2) * solid_temperature(a, x, r) - t_here;
  const NodeAddr<kMode> n = node_addr<St, kMode>(x, r, a.lx, row_b);
  C g[9];
  pull_thermal<St, kMode>(a, src, n, lm, plane_b, row_b, x, r, g);
  C t = sum9(g);
  if constexpr (St::kDev) t += a.ref_t;
  return t;
}

// ---------------------------------------------------------------- kernel
template <class St, int BX, unsigned kMode>
__global__ __launch_bounds__(BX)
#if defined(TLB_WAVES_PER_EU)
__attribute__((amdgpu_waves_per_eu(TLB_WAVES_PER_EU)))
#endif
void lb_step_kernel(StepArgs<typename St::C> a) {
  using C = typename St::C;
  using T = typename St::T;
  using O = Off<kMode>;
  constexpr bool kTauOne = (kMode & kModeTauOne) != 0;
  constexpr int kKept = kTauOne ? 4 : 18;  // values kept per pulled row
  constexpr int W = BX + 4;   // ring row width: strip plus 2 halo columns each side
  constexpr int R = 6;        // ring rows
  __shared__ C s_rho[2][R][W];
  __shared__ C s_psi[2][R][W];

  const void* src = a.src;
  void* dst = a.dst;
  const int lx = a.lx, ly = a.ly;
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * BX;
  const int y0 = blockIdx.y * a.rows_per_block;
  const int y1 = min(y0 + a.rows_per_block, ly);
  const O row_b = (O)a.pitch * sizeof(T);
  const O plane_b = (O)a.pop_stride * sizeof(T);

  // own column (idle threads of a ragged strip still fill their ring slot,
  // with a wrapped column, so the halo of the last valid column is right)
  const int xo = x0 + tid;
  const bool own_valid = xo < lx;
  const int xw = xo % lx;

  // halo slots 0, 1, BX+2, BX+3: lanes 0..3 of one wavefront, taken in turn
  // by the block's wavefronts from row to row (a single divergent pass per
  // row instead of one per wavefront)
  constexpr int kWaves = BX / 64;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int hslot = lane < 2 ? lane : BX + lane;
  const int hx = ((x0 - 2 + hslot) % lx + lx) % lx;

  const C psi_w0 = psi_exp(a.rho_wall0, a.rho0, a.inv_rho0);
  const C psi_w1 = psi_exp(a.rho_wall1, a.rho0, a.inv_rho0);

  double acc[7] = {0, 0, 0, 0, 0, 0, 0};

  // Densities of node (x, r) into ring slot `slot` / column `col`; the pulled
  // populations land in f and the node's link mask in lm. Returns whether
  // the node was pulled (fluid, inside the lattice).
  auto density = [&](int x, int r, int slot, int col, C (&f)[18], uint32_t& lm) {
    C ra = a.rho_wall0, rb = a.rho_wall1, pa = psi_w0, pb = psi_w1;
    bool pulled = false;
    lm = kSelfSolid;
    if (r >= 0 && r < ly) {
      lm = link_mask<kMode>(a, x, r);
      if (!((kMode & kModeSolid) != 0 && (lm & kSelfSolid))) {
        const NodeAddr<kMode> n = node_addr<St, kMode>(x, r, lx, row_b);
        pull_fluid<St, kMode>(src, n, lm, plane_b, row_b, f);
        ra = sum9(f);
        rb = sum9(f + 9);
        if constexpr (St::kDev) {
          ra += a.ref_a;
          rb += a.ref_b;
        }
        pa = psi_exp(ra, a.rho0, a.inv_rho0);
        pb = psi_exp(rb, a.rho0, a.inv_rho0);
        pulled = true;
      }
    }
    s_rho[0][slot][col] = ra;
    s_rho[1][slot][col] = rb;
    s_psi[0][slot][col] = pa;
    s_psi[1][slot][col] = pb;
    return pulled;
  };

  // One row iteration: pull row r = y0 - 2 + k (kept in kw/lw) and complete
  // row y = r - 2 from ku/lu (kept two iterations earlier). The g values of
  // row y are pulled together with the f values of row r, so each
  // iteration waits on memory once. With tau = tau_g = 1 the collision
  // returns the equilibria, so a kept row is only its moments.
  auto iterate = [&](int k, C (&kw)[kKept], uint32_t& lw, const C (&ku)[kKept], uint32_t lu) {
    const int r = y0 - 2 + k;
    const int y = r - 2;
    const int slot = k % R;
    const bool out = k >= 4 && y < y1 && own_valid;
    const bool out_fluid = out && !((kMode & kModeSolid) != 0 && (lu & kSelfSolid));
    const NodeAddr<kMode> n = node_addr<St, kMode>(xw, y < 0 ? 0 : y, lx, row_b);
    C g[9];
    if (out_fluid) pull_thermal<St, kMode>(a, src, n, lu, plane_b, row_b, xw, y, g);
    {
      C f[18];
      const bool pulled = density(xw, r, slot, tid + 2, f, lw);
      if constexpr (kTauOne) {
        if (pulled) {
          kw[0] = sum9(f);
          kw[1] = sum9(f + 9);
          kw[2] = momentum_x(f, f + 9);
          kw[3] = momentum_y(f, f + 9);
        }
      } else {
#pragma unroll
        for (int i = 0; i < 18; ++i) kw[i] = f[i];
      }
    }
    if (wave == k % kWaves && lane < 4) {
      C hf[18];
      uint32_t hl;
      density(hx, r, slot, hslot, hf, hl);
    }
    __syncthreads();

    if (!out) return;
    if (!out_fluid) {
      if constexpr ((kMode & kModeStore) != 0) {
#pragma unroll
        for (int p = 0; p < 27; ++p) st<St, kMode>(dst, (O)p * plane_b + n.own, C(0));
      }
      if constexpr ((kMode & kModeFields) != 0) {
        const size_t nn = (size_t)lx * ly, q = (size_t)y * lx + xo;
        a.fields[q] = (double)a.rho_wall0;
        a.fields[nn + q] = (double)a.rho_wall1;
        a.fields[2 * nn + q] = 0.0;
        a.fields[3 * nn + q] = 0.0;
        a.fields[4 * nn + q] = (double)solid_temperature(a, xo, y);
      }
      return;
    }
    [[maybe_unused]] const C* fa = ku;
    [[maybe_unused]] const C* fb = ku + 9 * (kTauOne ? 0 : 1);
    // ---- moments: stored-form sums (exact for the fixed-point storage)
    C Da, Db, jx, jy;
    if constexpr (kTauOne) {
      Da = ku[0];
      Db = ku[1];
      jx = ku[2];
      jy = ku[3];
    } else {
      Da = sum9(fa);
      Db = sum9(fb);
      jx = momentum_x(fa, fb);
      jy = momentum_y(fa, fb);
    }
    C ra = Da, rb = Db;
    if constexpr (St::kDev) {
      ra += a.ref_a;
      rb += a.ref_b;
    }
    const C Dt = sum9(g);
    C temp = Dt;
    if constexpr (St::kDev) temp += a.ref_t;

    // ---- forces from the ring (rows y-2..y+2 are slots k-4..k)
    const int s0 = tid + 2;
    int rs[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) rs[d] = (k + 2 + d) % R;  // d = dy + 2
    C FA[2], FB[2];
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      C ax = 0, ay = 0, qx = 0, qy = 0;  // NN sums (w), 25-point sums (p)
#pragma unroll
      for (int dy = -2; dy <= 2; ++dy) {
#pragma unroll
        for (int dx = 1; dx <= 2; ++dx) {
          const int c2 = dx * dx + dy * dy;
          const C diff = s_psi[l][rs[dy + 2]][s0 + dx] - s_psi[l][rs[dy + 2]][s0 - dx];
          qx += (p_c2<C>(c2) * C(dx)) * diff;
          if (c2 <= 2) ax += (w_c2<C>(c2) * C(dx)) * diff;
        }
      }
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) {
#pragma unroll
        for (int dy = 1; dy <= 2; ++dy) {
          const int c2 = dx * dx + dy * dy;
          const C diff = s_psi[l][rs[dy + 2]][s0 + dx] - s_psi[l][rs[2 - dy]][s0 + dx];
          qy += (p_c2<C>(c2) * C(dy)) * diff;
          if (c2 <= 2) ay += (w_c2<C>(c2) * C(dy)) * diff;
        }
      }
      const C psi_here = s_psi[l][rs[2]][s0];
      const C ga = l == 0 ? a.ga0 : a.ga1;
      const C gr = l == 0 ? a.gr0 : a.gr1;
      C* F = l == 0 ? FA : FB;
      F[0] = -psi_here * (ga * ax + gr * qx);
      F[1] = -psi_here * (ga * ay + gr * qy);
    }
    // cross force (NN, w, psi = rho / rho0): acts on l from the other one
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const int m = 1 - l;
      C sx = 0, sy = 0;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        const int c2 = 1 + dy * dy;
        sx += w_c2<C>(c2) * (s_rho[m][rs[dy + 2]][s0 + 1] - s_rho[m][rs[dy + 2]][s0 - 1]);
      }
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int c2 = 1 + dx * dx;
        sy += w_c2<C>(c2) * (s_rho[m][rs[3]][s0 + dx] - s_rho[m][rs[1]][s0 + dx]);
      }
      const C rl = l == 0 ? ra : rb;
      const C pre = -a.g12 * rl * a.inv_rho0 * a.inv_rho0;
      C* F = l == 0 ? FA : FB;
      F[0] += pre * sx;
      F[1] += pre * sy;
    }
    // buoyancy (Eq. (22))
    FA[1] += ra * a.alpha_g * temp;
    FB[1] += rb * a.alpha_g * temp;

    // ---- velocities
    const C rho = ra + rb;
    const C inv_rho = C(1) / rho;
    const C ux = jx * inv_rho, uy = jy * inv_rho;
    const C Fx = FA[0] + FB[0], Fy = FA[1] + FB[1];
    const C hx = ux + C(0.5) * Fx * inv_rho;
    const C hy = uy + C(0.5) * Fy * inv_rho;

    if constexpr ((kMode & kModeStore) != 0) {
      const C tA = a.tau / ra, tB = a.tau / rb;
      const C uax = ux + FA[0] * tA, uay = uy + FA[1] * tA;
      const C ubx = ux + FB[0] * tB, uby = uy + FB[1] * tB;
      const C ua2 = uax * uax + uay * uay;
      const C ub2 = ubx * ubx + uby * uby;
      const C uh2 = hx * hx + hy * hy;
      // BGK relaxation written as f^eq + (1 - 1/tau)(f - f^eq) in stored
      // form (exactly f^eq at tau = 1). The rest population takes the
      // remainder of the zeroth moment, so the stored populations sum to
      // rho (and T) up to unbiased rounding (exactly for fixed point): the
      // weights rounded to the storage type do not sum to 1 and would
      // otherwise create or destroy mass at every collision.
      const C ka = C(1) - a.inv_tau, kg = C(1) - a.inv_tau_g;
      C sa = 0, sb = 0, sg = 0;
      const O p9 = plane_b * 9, p18 = plane_b * 18;
#define TLB_COLLIDE(I)                                                                 \
  {                                                                                    \
    constexpr int cx = Dir<I>::cx, cy = Dir<I>::cy;                                   \
    constexpr C w = w_dir<C>(I);                                                       \
    const C cua = C(cx) * uax + C(cy) * uay;                                           \
    const C cub = C(cx) * ubx + C(cy) * uby;                                           \
    const C cuh = C(cx) * hx + C(cy) * hy;                                             \
    C ea = w * ra * (C(1) + C(3) * cua + C(4.5) * cua * cua - C(1.5) * ua2);           \
    C eb = w * rb * (C(1) + C(3) * cub + C(4.5) * cub * cub - C(1.5) * ub2);           \
    C eg = w * temp * (C(1) + C(3) * cuh + C(4.5) * cuh * cuh - C(1.5) * uh2);         \
    if constexpr (St::kDev) {                                                          \
      ea -= w * a.ref_a;                                                               \
      eb -= w * a.ref_b;                                                               \
      eg -= w * a.ref_t;                                                               \
    }                                                                                  \
    C qa = ea, qb = eb, qg = eg;                                                       \
    if constexpr (!kTauOne) {                                                          \
      qa += ka * (fa[I] - ea);                                                         \
      qb += ka * (fb[I] - eb);                                                         \
      qg += kg * (g[I] - eg);                                                          \
    }                                                                                  \
    qa = St::grid(qa);                                                                 \
    qb = St::grid(qb);                                                                 \
    qg = St::grid(qg);                                                                 \
    if constexpr (St::kFix) {                                                          \
      sa += qa;                                                                        \
      sb += qb;                                                                        \
      sg += qg;                                                                        \
    } else {                                                                           \
      sa += ea;                                                                        \
      sb += eb;                                                                        \
      sg += eg;                                                                        \
    }                                                                                  \
    const O o = (O)I * plane_b + n.own;                                                \
    st<St, kMode>(dst, o, qa);                                                         \
    st<St, kMode>(dst, o + p9, qb);                                                    \
    st<St, kMode>(dst, o + p18, qg);                                                   \
  }
      TLB_COLLIDE(1) TLB_COLLIDE(2) TLB_COLLIDE(3) TLB_COLLIDE(4)
      TLB_COLLIDE(5) TLB_COLLIDE(6) TLB_COLLIDE(7) TLB_COLLIDE(8)
#undef TLB_COLLIDE
      if constexpr (St::kFix) {
        // exact remainders: the stored populations sum to the pulled ones
        st<St, kMode>(dst, n.own, St::grid(Da - sa));
        st<St, kMode>(dst, n.own + p9, St::grid(Db - sb));
        st<St, kMode>(dst, n.own + p18, St::grid(Dt - sg));
      } else if constexpr (kTauOne) {
        st<St, kMode>(dst, n.own, Da - sa);
        st<St, kMode>(dst, n.own + p9, Db - sb);
        st<St, kMode>(dst, n.own + p18, Dt - sg);
      } else {
        const C ea = Da - sa, eb = Db - sb, eg = Dt - sg;
        st<St, kMode>(dst, n.own, ea + ka * (fa[0] - ea));
        st<St, kMode>(dst, n.own + p9, eb + ka * (fb[0] - eb));
        st<St, kMode>(dst, n.own + p18, eg + kg * (g[0] - eg));
      }
    }
    // FP64 densities for output: reference plus the stored-form sum
    const double dra = St::kDev ? (double)a.ref_a + (double)Da : (double)ra;
    const double drb = St::kDev ? (double)a.ref_b + (double)Db : (double)rb;
    const double dtt = St::kDev ? (double)a.ref_t + (double)Dt : (double)temp;
    if constexpr ((kMode & kModeFields) != 0) {
      const size_t nn = (size_t)lx * ly, q = (size_t)y * lx + xo;
      a.fields[q] = dra;
      a.fields[nn + q] = drb;
      a.fields[2 * nn + q] = (double)hx;
      a.fields[3 * nn + q] = (double)hy;
      a.fields[4 * nn + q] = dtt;
    }
    if constexpr ((kMode & kModeObserve) != 0) {
      const C tn = neighbour_temperature<St, kMode>(a, src, xw, y + 1, temp, plane_b, row_b);
      const C ts = neighbour_temperature<St, kMode>(a, src, xw, y - 1, temp, plane_b, row_b);
      acc[0] += dra;
      acc[1] += drb;
      acc[2] += dtt;
      acc[3] += (double)hy * dtt;
      acc[4] += 0.5 * ((double)tn - (double)ts);
      acc[5] += (double)hx * (double)hx + (double)hy * (double)hy;
      if (y == ly - 1) acc[6] += dtt - (double)a.t_top;
    }
  };

  // Three sets of kept rows; the unrolled loop rotates their roles. The
  // iteration count is rounded up to a multiple of 3: the extra iterations
  // only pull in-range rows (or ghost rows) and complete nothing.
  C f0[kKept], f1[kKept], f2[kKept];
  uint32_t l0 = 0, l1 = 0, l2 = 0;
  const int n_iter = ((y1 - y0) + 4 + 2) / 3 * 3;
  for (int k = 0; k < n_iter; k += 3) {
    iterate(k, f0, l0, f1, l1);
    iterate(k + 1, f1, l1, f2, l2);
    iterate(k + 2, f2, l2, f0, l0);
  }

  if constexpr ((kMode & kModeObserve) != 0) {
    // block reduction of the 7 sums in a fixed order (deterministic)
    __shared__ double s_acc[BX / 64][8];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      double v = acc[j];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
      if ((tid & 63) == 0) s_acc[tid >> 6][j] = v;
    }
    __syncthreads();
    if (tid < 7) {
      double v = 0;
      for (int w = 0; w < BX / 64; ++w) v += s_acc[w][tid];
      a.partials[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 8 + tid] = v;
    }
  }
}

// Equilibrium start state f(0) = f^eq(rho_l, u0), g(0) = g^eq(T, u0) written
// at each node (the init variant of the step kernel reads it in place).
template <class St>
__global__ __launch_bounds__(256) void lb_init_equilibrium(
    typename St::T* __restrict__ buf, const double* __restrict__ rho_a,
    const double* __restrict__ rho_b, const double* __restrict__ temp,
    const double* __restrict__ ux0, const double* __restrict__ uy0,
    const uint8_t* __restrict__ solid, int lx, int ly, int pitch, long long pop_stride,
    typename St::C ref_a, typename St::C ref_b, typename St::C ref_t) {
  using C = typename St::C;
  const C ref[3] = {St::kDev ? ref_a : C(0), St::kDev ? ref_b : C(0), St::kDev ? ref_t : C(0)};
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= lx) return;
  const size_t q = (size_t)y * lx + x;
  const long long off = (long long)y * pitch + x;
  const bool is_solid = solid != nullptr && solid[q] != 0;
  const C ux = ux0 ? (C)ux0[q] : C(0), uy = uy0 ? (C)uy0[q] : C(0);
  const C u2 = ux * ux + uy * uy;
  const C dens[3] = {(C)rho_a[q], (C)rho_b[q], (C)temp[q]};
  C sum[3] = {C(0), C(0), C(0)};
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const C cu = C(dir_cx(i)) * ux + C(dir_cy(i)) * uy;
    const C shape = w_dir<C>(i) * (C(1) + C(3) * cu + C(4.5) * cu * cu - C(1.5) * u2);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const C v = dens[s] * shape;
      const C d = St::grid(v - w_dir<C>(i) * ref[s]);   // stored form
      sum[s] += St::kFix ? d : v;
      St::store(buf + (long long)(i + 9 * s) * pop_stride + off, is_solid ? C(0) : d);
    }
  }
  // rest population: zeroth moment minus the other eight (exact mass)
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const C d = St::kFix ? St::grid(St::grid(dens[s] - ref[s]) - sum[s])
                         : (dens[s] - sum[s]) - w_dir<C>(0) * ref[s];
    St::store(buf + (long long)(9 * s) * pop_stride + off, is_solid ? C(0) : d);
  }
}

// Copy populations out as doubles [27][ly][lx] (drops the row padding, adds
// the deviation references back, zero at solid nodes).
template <class St>
__global__ __launch_bounds__(256) void lb_export_populations(
    const typename St::T* __restrict__ buf, double* __restrict__ out,
    const uint8_t* __restrict__ solid, int lx, int ly, int pitch, long long pop_stride,
    typename St::C ref_a, typename St::C ref_b, typename St::C ref_t) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int p = blockIdx.z;
  if (x >= lx) return;
  double v = (double)St::load(buf + p * pop_stride + (long long)y * pitch + x);
  if constexpr (St::kDev)
    v += w_dir<double>(p % 9) * (double)(p < 9 ? ref_a : (p < 18 ? ref_b : ref_t));
  if (solid[(size_t)y * lx + x] != 0) v = 0.0;
  out[((size_t)p * ly + y) * lx + x] = v;
}

}  // namespace tlbk
