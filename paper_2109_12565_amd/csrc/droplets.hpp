// Droplet detection on the GPU (Sec. 2.4) and the droplet Nusselt number
// (Sec. 3.3.2 Eq. (25)).
//
// A droplet is a 4-connected cluster of fluid nodes whose density of the
// first component exceeds the bulk threshold B_th (x periodic). Clusters are
// found by a lock-free union-find: every node starts as its own parent, each
// bulk node unites with its bulk neighbours to the right (periodic) and
// above, linking the larger root under the smaller one with an atomic
// minimum, and a final pass points every node at its root. The root of a
// cluster is therefore its smallest node index, and droplets are numbered in
// the order of their roots (canonical, independent of scheduling).
//
// The unions run in two passes: each block first unites the links inside its
// 64 x 16 tile in LDS and writes, for every bulk node, the smallest index of
// its cluster within the tile; a global pass then unites only the links that
// cross a tile edge (or the periodic seam), so most unions never touch
// global memory.
//
// Per-droplet sums (node count, sum rho_A, sum rho_A X, sum rho_A Y) are
// exact: each term is rounded once to a multiple of 2^-40 and split into a
// high and a low 32-bit part; the parts are summed as 64-bit integers, first
// over the lanes of a wavefront that belong to the same droplet and then
// across wavefronts with integer atomics, so the result does not depend on
// the order of the additions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tlbk {

// One droplet as the C ABI returns it (struct tlb_droplet).
struct DropRecord {
  int64_t root, size;
  double mass, x, y, nu;
};

struct DropArgs {
  const double* fields;     // [5][ly][lx]: rho_A, rho_B, u^H_x, u^H_y, T
  const uint8_t* solid;     // [ly*lx]
  const double* t_bottom;   // [lx] (FP64 copy)
  int32_t* parent;          // [ly*lx] union-find parents, -1 outside droplets
  int32_t* rid;             // [ly*lx] droplet number of each root
  int32_t* block_count;     // [nblocks] roots per block, then exclusive offsets
  int64_t* acc;             // [count][7] size, mass hi/lo, mx hi/lo, my hi/lo
  int64_t* roots;           // [count] root node of each droplet
  DropRecord* out;          // [count]
  int32_t* label;           // [ly*lx] droplet number, -1 outside
  int* error;               // set when a bounded loop runs out
  const int32_t* total;     // droplet count (written by drop_scan_tiles)
  double threshold, t_top, kappa, dt_nominal;
  int lx, ly, n;
  int capacity;             // droplets acc, roots and out have room for; the
                            // droplets beyond it are numbered but not summed
};

constexpr int kDropItems = 16;                 // nodes per thread in the counting passes
constexpr int kDropTile = 256 * kDropItems;    // nodes per block in the counting passes

__device__ inline int32_t load_parent(const int32_t* p, int q) {
  return __hip_atomic_load(p + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of q, halving the path on the way (q is pointed at its grandparent,
// still an ancestor in its cluster). Parents only ever decrease and
// parent[q] <= q, so the walk strictly descends: at most n steps (`cap`);
// running out sets the error flag instead of looping on.
__device__ inline int32_t find_root(int32_t* parent, int32_t q, int cap, int* error) {
  for (int it = 0; it < cap; ++it) {
    const int32_t p = load_parent(parent, q);
    if (p == q) return q;
    const int32_t g = load_parent(parent, p);
    if (g == p) return p;
    atomicMin(parent + q, g);
    q = g;
  }
  atomicOr(error, 1);
  return q;
}

// Unite the clusters of a and b (both bulk nodes). An atomic minimum links
// the larger root under the smaller; if that node was no longer a root, the
// walk continues from the parent it had (a strictly smaller index).
__device__ inline void unite(int32_t* parent, int32_t a, int32_t b, int cap, int* error) {
  for (int it = 0; it < cap; ++it) {
    a = find_root(parent, a, cap, error);
    b = find_root(parent, b, cap, error);
    if (a == b) return;
    if (a < b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    const int32_t old = atomicMin(parent + a, b);
    if (old == a) return;
    a = old;
  }
  atomicOr(error, 1);
}

__device__ inline bool is_bulk(const DropArgs& a, int q) {
  return a.solid[q] == 0 && a.fields[q] > a.threshold;
}

// Tile of the LDS union pass: 64 columns x 16 rows, 4 nodes per thread.
constexpr int kLocalW = 64, kLocalH = 16, kLocalN = kLocalW * kLocalH;

__device__ inline int lds_parent(const int* p, int i) {
  return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// find_root / unite on a tile's LDS parents (local indices, row-major in the
// tile; bounded walks as in the global ones).
__device__ inline int lds_find(int* par, int q, bool& fail) {
  for (int it = 0; it <= kLocalN; ++it) {
    const int p = lds_parent(par, q);
    if (p == q) return q;
    const int g = lds_parent(par, p);
    if (g == p) return p;
    atomicMin(par + q, g);
    q = g;
  }
  fail = true;
  return q;
}

__device__ inline void lds_unite(int* par, int a, int b, bool& fail) {
  for (int it = 0; it <= kLocalN; ++it) {
    a = lds_find(par, a, fail);
    b = lds_find(par, b, fail);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(par + a, b);
    if (old == a) return;
    a = old;
  }
  fail = true;
}

// Union pass inside each tile. Local row-major order is the global order
// restricted to the tile, so a tile cluster's local root is its smallest
// node index, which becomes the parent of every node of the cluster.
__global__ __launch_bounds__(256) void drop_local(DropArgs a) {
  __shared__ int par[kLocalN];
  const int x0 = blockIdx.x * kLocalW, y0 = blockIdx.y * kLocalH;
  for (int k = 0; k < kLocalN / 256; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int gx = x0 + (i % kLocalW), gy = y0 + i / kLocalW;
    const bool bulk = gx < a.lx && gy < a.ly && is_bulk(a, gy * a.lx + gx);
    par[i] = bulk ? i : -1;
  }
  __syncthreads();
  bool fail = false;
  for (int k = 0; k < kLocalN / 256; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (lds_parent(par, i) < 0) continue;
    const int lxi = i % kLocalW, lyi = i / kLocalW;
    if (lxi + 1 < kLocalW && x0 + lxi + 1 < a.lx && lds_parent(par, i + 1) >= 0)
      lds_unite(par, i, i + 1, fail);
    if (lyi + 1 < kLocalH && y0 + lyi + 1 < a.ly && lds_parent(par, i + kLocalW) >= 0)
      lds_unite(par, i, i + kLocalW, fail);
  }
  __syncthreads();
  for (int k = 0; k < kLocalN / 256; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int gx = x0 + (i % kLocalW), gy = y0 + i / kLocalW;
    if (gx >= a.lx || gy >= a.ly) continue;
    int out = -1;
    if (lds_parent(par, i) >= 0) {
      const int r = lds_find(par, i, fail);
      out = (y0 + r / kLocalW) * a.lx + x0 + r % kLocalW;
    }
    a.parent[gy * a.lx + gx] = out;
  }
  if (fail) atomicOr(a.error, 1);
}

// Global union pass over the links the tiles did not cover: from a tile's
// last column (or the lattice's, across the periodic seam) to the right, and
// from a tile's top row upwards.
// Threads of drop_union_border: one per node of a tile's last column
// (its right link; the last tile's is the periodic seam), then one per
// node of a tile's last row below the top row (its upper link).
__host__ __device__ inline int border_columns(int lx) { return (lx + kLocalW - 1) / kLocalW; }
__host__ __device__ inline int border_rows(int ly) { return (ly - 1) / kLocalH; }
__host__ __device__ inline long long border_links(int lx, int ly) {
  return (long long)border_columns(lx) * ly + (long long)border_rows(ly) * lx;
}

__global__ __launch_bounds__(256) void drop_union_border(DropArgs a) {
  long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long nv = (long long)border_columns(a.lx) * a.ly;
  if (e < nv) {
    const int k = (int)(e / a.ly), y = (int)(e - (long long)k * a.ly);
    const int x = min((k + 1) * kLocalW, a.lx) - 1;
    const int q = y * a.lx + x;
    const int right = y * a.lx + (x + 1 == a.lx ? 0 : x + 1);
    if (right != q && a.parent[q] >= 0 && a.parent[right] >= 0)
      unite(a.parent, q, right, a.n + 1, a.error);
    return;
  }
  e -= nv;
  if (e >= (long long)border_rows(a.ly) * a.lx) return;
  const int r = (int)(e / a.lx), x = (int)(e - (long long)r * a.lx);
  const int y = (r + 1) * kLocalH - 1;  // below ly - 1
  const int q = y * a.lx + x;
  if (a.parent[q] >= 0 && a.parent[q + a.lx] >= 0) unite(a.parent, q, q + a.lx, a.n + 1, a.error);
}

// Roots per tile of kDropTile nodes.
__global__ __launch_bounds__(256) void drop_count_roots(DropArgs a) {
  __shared__ int s[256];
  const int base = blockIdx.x * kDropTile + threadIdx.x * kDropItems;
  int c = 0;
  for (int j = 0; j < kDropItems; ++j) {
    const int q = base + j;
    if (q < a.n && a.parent[q] == q) ++c;
  }
  s[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.block_count[blockIdx.x] = s[0];
}

// Exclusive scan of the tile counts (one block); block_count[nblocks] gets
// the total.
__global__ __launch_bounds__(256) void drop_scan_tiles(int32_t* count, int nblocks) {
  __shared__ int s[256];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nblocks; b0 += 256) {
    const int i = b0 + threadIdx.x;
    const int v = i < nblocks ? count[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele scan
      const int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nblocks) count[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 255) carry += s[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) count[nblocks] = carry;
}

// Droplet number of every root: tile offset plus the rank within the tile.
__global__ __launch_bounds__(256) void drop_number_roots(DropArgs a) {
  __shared__ int s[256];
  const int base = blockIdx.x * kDropTile + threadIdx.x * kDropItems;
  int c = 0;
  for (int j = 0; j < kDropItems; ++j) {
    const int q = base + j;
    if (q < a.n && a.parent[q] == q) ++c;
  }
  s[threadIdx.x] = c;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int id = a.block_count[blockIdx.x] + s[threadIdx.x] - c;
  for (int j = 0; j < kDropItems; ++j) {
    const int q = base + j;
    if (q < a.n && a.parent[q] == q) {
      a.rid[q] = id;
      if (id < a.capacity) a.roots[id] = q;
      ++id;
    }
  }
}

// Fixed-point term: v rounded to a multiple of 2^-40, split into a high
// part (multiples of 2^-8) and a low part in [0, 2^32) units of 2^-40.
__device__ inline void split_fixed(double v, int64_t& hi, int64_t& lo) {
  const int64_t f = __double2ll_rn(v * 1099511627776.0);  // 2^40
  hi = f >> 32;
  lo = f - (hi << 32);
}

__device__ inline double fixed_value(int64_t hi, int64_t lo) {
  return ((double)hi * 4294967296.0 + (double)lo) * (1.0 / 1099511627776.0);
}

// Per node: its droplet number, and its terms of the droplet's sums (x
// taken within half a period of the root's x). A block sums a tile of
// kLocalW columns x kAccRows rows: each thread walks kAccRun rows of one
// column (a wavefront reads one row at a time) and keeps the running sums
// of the droplet it is in; when the droplet changes it adds them to the
// droplet's slot of an LDS table (open addressing on the droplet number).
// At the end each slot issues one set of global atomics; a run that finds
// the table full adds to global memory directly. The sums are integers,
// so the result does not depend on the order.
constexpr int kAccSlots = 128;
constexpr int kAccRun = 16;
constexpr int kAccRows = kAccRun * (256 / kLocalW);

__device__ inline void acc_flush(DropArgs& a, int32_t* key, unsigned long long (*val)[7], int d,
                                 const int64_t (&sum)[7]) {
  int slot = d & (kAccSlots - 1), found = -1;
  for (int probe = 0; probe < kAccSlots; ++probe) {
    const int32_t old = atomicCAS(&key[slot], -1, d);
    if (old == -1 || old == d) {
      found = slot;
      break;
    }
    slot = (slot + 1) & (kAccSlots - 1);
  }
  if (found >= 0) {
#pragma unroll
    for (int j = 0; j < 7; ++j) atomicAdd(&val[found][j], (unsigned long long)sum[j]);
  } else {
    unsigned long long* c = reinterpret_cast<unsigned long long*>(a.acc + (size_t)d * 7);
#pragma unroll
    for (int j = 0; j < 7; ++j) atomicAdd(c + j, (unsigned long long)sum[j]);
  }
}

__global__ __launch_bounds__(256) void drop_accumulate(DropArgs a) {
  __shared__ int32_t key[kAccSlots];
  __shared__ unsigned long long val[kAccSlots][7];
  for (int i = threadIdx.x; i < kAccSlots; i += 256) {
    key[i] = -1;
#pragma unroll
    for (int j = 0; j < 7; ++j) val[i][j] = 0;
  }
  __syncthreads();
  const int x = blockIdx.x * kLocalW + (threadIdx.x % kLocalW);
  const int ys = blockIdx.y * kAccRows + (threadIdx.x / kLocalW) * kAccRun;
  int cur = -1;  // droplet of the running sums
  int64_t sum[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < kAccRun; ++k) {
    const int y = ys + k;
    if (x >= a.lx || y >= a.ly) break;
    const int q = y * a.lx + x;
    // the cluster root (the walk halves the path, as in unite)
    const int32_t root = a.parent[q] >= 0 ? find_root(a.parent, q, a.n + 1, a.error) : -1;
    const int lab = root >= 0 ? a.rid[root] : -1;
    a.label[q] = lab;
    const int d = lab < a.capacity ? lab : -1;  // droplets beyond the room: not summed
    if (d != cur) {
      if (cur >= 0) acc_flush(a, key, val, cur, sum);
      cur = d;
#pragma unroll
      for (int j = 0; j < 7; ++j) sum[j] = 0;
    }
    if (d >= 0) {
      const int xr = root % a.lx, yr = root / a.lx;
      double dx = (double)(x - xr);
      if (dx > 0.5 * a.lx) dx -= a.lx;
      if (dx < -0.5 * a.lx) dx += a.lx;
      const double r = a.fields[q];
      int64_t t[7];
      t[0] = 1;
      split_fixed(r, t[1], t[2]);
      split_fixed(r * ((double)xr + dx), t[3], t[4]);
      split_fixed(r * (double)(yr + (y - yr)), t[5], t[6]);
#pragma unroll
      for (int j = 0; j < 7; ++j) sum[j] += t[j];
    }
  }
  if (cur >= 0) acc_flush(a, key, val, cur, sum);
  __syncthreads();
  for (int i = threadIdx.x; i < kAccSlots; i += 256) {
    const int32_t dl = key[i];
    if (dl < 0) continue;
    unsigned long long* c = reinterpret_cast<unsigned long long*>(a.acc + (size_t)dl * 7);
#pragma unroll
    for (int j = 0; j < 7; ++j) atomicAdd(c + j, val[i][j]);
  }
}

// FP64 copy of the bottom wall temperature (the handle keeps the compute
// type of its storage); also clears the error flag of the union passes,
// which run after it.
__global__ __launch_bounds__(256) void drop_bottom_temperature(const void* src, int src_is_f32,
                                                               double* dst, int lx, int* error) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x == 0) *error = 0;
  if (x >= lx) return;
  dst[x] = src_is_f32 ? (double)static_cast<const float*>(src)[x]
                      : static_cast<const double*>(src)[x];
}

// Zero the first `*count` droplet accumulators (the count is read on the
// device; the grid covers `max_count`).
__global__ __launch_bounds__(256) void drop_clear(int64_t* acc, const int32_t* count,
                                                  int max_count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int c = *count;
  if (i >= max_count || i >= c) return;
#pragma unroll
  for (int j = 0; j < 7; ++j) acc[(size_t)i * 7 + j] = 0;
}

// Temperature gradient dT/dy at node (x, y) by central differences with
// the mirror value 2 T_w - T at a solid neighbour (0 at solid nodes).
__device__ inline double node_dtdy(const DropArgs& a, int x, int y) {
  const size_t nn = (size_t)a.lx * a.ly;
  const double* T = a.fields + 4 * nn;
  const int q = y * a.lx + x;
  if (a.solid[q] != 0) return 0.0;
  const double t = T[q];
  double tn, ts;
  if (y + 1 >= a.ly) tn = 2.0 * a.t_top - t;
  else if (a.solid[q + a.lx] != 0) tn = 2.0 * T[q + a.lx] - t;
  else tn = T[q + a.lx];
  if (y - 1 < 0) ts = 2.0 * a.t_bottom[x] - t;
  else if (a.solid[q - a.lx] != 0) ts = 2.0 * T[q - a.lx] - t;
  else ts = T[q - a.lx];
  return 0.5 * (tn - ts);
}

// Per droplet: centre of mass, and Eq. (25) with u^H_y, T and dT/dy
// interpolated bilinearly at the centre (x periodic, y clamped).
__global__ __launch_bounds__(256) void drop_finalize(DropArgs a) {
  const int d = blockIdx.x * 256 + threadIdx.x;
  if (d >= *a.total || d >= a.capacity) return;
  const int64_t* c = a.acc + (size_t)d * 7;
  const double m = fixed_value(c[1], c[2]);
  double X = fixed_value(c[3], c[4]) / m;
  double Y = fixed_value(c[5], c[6]) / m;
  X = fmod(X, (double)a.lx);
  if (X < 0) X += a.lx;
  const double yc = Y < 0 ? 0.0 : (Y > a.ly - 1 ? (double)(a.ly - 1) : Y);
  int x0 = (int)floor(X), y0 = (int)floor(yc);
  const double ax = X - x0, ay = yc - y0;
  int x1 = x0 + 1, y1 = y0 + 1;
  x0 %= a.lx;
  x1 %= a.lx;
  if (y1 > a.ly - 1) y1 = a.ly - 1;
  const size_t nn = (size_t)a.lx * a.ly;
  const double* uy = a.fields + 3 * nn;
  const double* T = a.fields + 4 * nn;
  const int q00 = y0 * a.lx + x0, q01 = y0 * a.lx + x1, q10 = y1 * a.lx + x0, q11 = y1 * a.lx + x1;
  const double w00 = (1 - ax) * (1 - ay), w01 = ax * (1 - ay), w10 = (1 - ax) * ay, w11 = ax * ay;
  const double u = w00 * uy[q00] + w01 * uy[q01] + w10 * uy[q10] + w11 * uy[q11];
  const double t = w00 * T[q00] + w01 * T[q01] + w10 * T[q10] + w11 * T[q11];
  const double g = w00 * node_dtdy(a, x0, y0) + w01 * node_dtdy(a, x1, y0) +
                   w10 * node_dtdy(a, x0, y1) + w11 * node_dtdy(a, x1, y1);
  DropRecord o;
  o.root = a.roots[d];
  o.size = c[0];
  o.mass = m;
  o.x = X;
  o.y = Y;
  o.nu = (u * t - a.kappa * g) / (a.kappa * a.dt_nominal / a.ly);
  a.out[d] = o;
}

}  // namespace tlbk
