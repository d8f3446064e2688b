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
// elements so every wavefront row access is aligned. Buffers below 4 GiB are
// accessed through a buffer resource: the plane and row part of an offset is
// uniform (a scalar register), the column part is per lane and fixed for
// the whole kernel, so the 27 loads and 27 stores of a node need no vector
// address arithmetic; kWide = true (4 GiB and above) adds 64-bit offsets to
// a flat pointer.
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
// point (kFix), where sums of stored values are exact; stored() is the value
// a store keeps (grid() for fixed point, the decoded 16-bit value for the
// floating formats). Stores are non-temporal: the next step reads the
// populations from HBM anyway.
//
// kRest32: the rest populations (planes 0, 9, 18) are kept in FP32, in
// three planes after the 27 16-bit ones, as the exact remainder of the
// node's zeroth moment minus its eight rounded moving populations. Sums of
// the stored values are then exact in FP32 (every 16-bit value and every
// remainder is a multiple of 2^-24 below 1 in magnitude), so the rounding
// of the moving populations moves no mass between nodes or components.
template <typename T_> struct Store {
  using T = T_;
  using C = T_;
  static constexpr bool kDev = false;
  static constexpr bool kFix = false;
  static constexpr bool kRest32 = false;
  static constexpr bool kFast = false;  // library expm1, IEEE division
  __device__ static C decode(T v) { return v; }
  __device__ static T encode(C v) { return v; }
  __device__ static C load(const T* p) { return decode(*p); }
  __device__ static void store(T* p, C v) { __builtin_nontemporal_store(encode(v), p); }
  __device__ static C grid(C v) { return v; }
  __device__ static C stored(C v) { return v; }
};

// 16-bit floating-point deviations, converted with round-to-nearest-even.
struct StoreF16Dev {
  using T = uint16_t;
  using C = float;
  static constexpr bool kDev = true;
  static constexpr bool kFix = false;
  static constexpr bool kRest32 = true;
  static constexpr bool kFast = true;   // cheaper psi and reciprocals
  __device__ static C grid(C v) { return v; }
  __device__ static C decode(T v) { return (float)__builtin_bit_cast(_Float16, v); }
  __device__ static T encode(C v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
  __device__ static C stored(C v) { return decode(encode(v)); }
  __device__ static C load(const T* p) { return decode(*p); }
  __device__ static void store(T* p, C v) { __builtin_nontemporal_store(encode(v), p); }
};

struct StoreBF16Dev {
  using T = uint16_t;
  using C = float;
  static constexpr bool kDev = true;
  static constexpr bool kFix = false;
  static constexpr bool kRest32 = true;
  static constexpr bool kFast = true;   // cheaper psi and reciprocals
  __device__ static C grid(C v) { return v; }
  __device__ static C decode(T v) { return __uint_as_float((uint32_t)v << 16); }
  __device__ static C stored(C v) { return decode(encode(v)); }
  __device__ static T encode(C v) {
    uint32_t u = __float_as_uint(v);
    const bool nan = (u & 0x7fffffffu) > 0x7f800000u;
    u += 0x7fffu + ((u >> 16) & 1u);  // round half to even on the dropped 16 bits
    return (uint16_t)(nan ? (__float_as_uint(v) >> 16) | 0x40u : u >> 16);
  }
  __device__ static C load(const T* p) { return decode(*p); }
  __device__ static void store(T* p, C v) { __builtin_nontemporal_store(encode(v), p); }
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
  static constexpr bool kRest32 = false;
  static constexpr bool kFast = true;   // cheaper psi and reciprocals
  static constexpr float kScale = 32768.0f;
  __device__ static C decode(T v) { return (float)v * (1.0f / kScale); }
  __device__ static T encode(C v) { return (int16_t)(int)(v * kScale); }  // v is on the grid
  __device__ static C load(const T* p) { return decode(*p); }
  __device__ static C grid(C v) {
    const float q = fminf(fmaxf(rintf(v * kScale), -32768.0f), 32767.0f);
    return q * (1.0f / kScale);
  }
  __device__ static C stored(C v) { return grid(v); }
  __device__ static void store(T* p, C v) { __builtin_nontemporal_store(encode(v), p); }
};

// ---------------------------------------------------------------- arguments
// Observable sums per block (FP64, fluid nodes): rho_A, rho_B, T, u^H_y T,
// |u^H|^2, and T - t_top over the top row.
constexpr int kObsSums = 6;

template <typename C>
struct StepArgs {
  const void* src;          // post-collision populations f*(t) (or f(0))
  void* dst;                // receives f*(t+1)
  void* moments;            // kModeMoments: [5][pop_stride] rho_A, rho_B, j_x, j_y, T of
                            // the pulled state, compute type (the fused kernel
                            // writes its second level at + 5 pop_stride)
  const uint16_t* link;     // [ly*lx] link masks (solid cells present only)
  const uint8_t* solid;     // [ly*lx] 0 fluid, 1 bottom-held, 2 top-held
  const C* t_bottom;        // [lx]
  double* partials;         // [gridDim.x*gridDim.y][kObsSums] observable sums
  double* fields;           // [5][ly][lx] rho_a, rho_b, ux, uy, T
  int lx, ly, pitch, rows_per_block;
  long long pop_stride;     // ly * pitch
  C inv_tau, inv_tau_g, tau, rho0, inv_rho0, g12;
  C ga0, ga1, gr0, gr1;
  C alpha_g, t_top, rho_wall0, rho_wall1;
  C ref_a, ref_b, ref_t;    // references of the 16-bit deviation storages
  C uw0, uw1;               // x-velocity of the bottom and top walls (kModeMoving)
};

// Kernel variants.
enum : unsigned {
  kModeInit = 1u,     // read f(0) at the node itself instead of pulling
  kModeStore = 2u,    // write f*(t+1)
  kModeObserve = 4u,  // accumulate observable sums into partials
  kModeFields = 8u,   // write the fields
  kModeSolid = 16u,   // solid cells present: use the link masks
  kModeWide = 32u,    // 64-bit byte offsets (population buffer >= 4 GiB)
  kModeTauOne = 64u,  // tau = tau_g = 1: the collision returns the equilibria
  kModeStress = 128u, // with kModeFields: also write the xy stress fields
  kModeMoving = 256u, // the flat walls move (momentum term in their bounce-back)
  kModeTopRow = 512u, // fused kernel: per-strip sums of T - t_top over the top row
                      // at both levels into partials (the taped run's loss terms)
  kModeMoments = 1024u // also write the moments of the pulled state (both
                       // levels in the fused kernel): the adjoint's tape at tau = 1
};

// rho0 (1 - exp(-rho/rho0)) of Eq. (12), evaluated as -rho0 expm1(-rho/rho0)
// to keep full relative precision at small rho (library expm1).
template <typename C> __device__ inline C psi_exp(C rho, C rho0, C inv_rho0) {
  return -rho0 * expm1(-rho * inv_rho0);
}
__device__ inline float psi_exp(float rho, float rho0, float inv_rho0) {
  return -rho0 * expm1f(-rho * inv_rho0);
}
// e^x - 1 for the 16-bit storages (whose rounding dominates any error
// here): its Taylor polynomial of degree 8 for |x| <= 1/2 (truncation below
// 1e-8 relative) and the hardware exp2 elsewhere, where 1 - e^x >= 0.39
// leaves no cancellation. About half the instructions of expm1f; FP32
// storage keeps the library function, whose errors do not share a sign.
__device__ inline float expm1_fast(float x) {
  float p = fmaf(x, 1.0f / 40320.0f, 1.0f / 5040.0f);
  p = fmaf(x, p, 1.0f / 720.0f);
  p = fmaf(x, p, 1.0f / 120.0f);
  p = fmaf(x, p, 1.0f / 24.0f);
  p = fmaf(x, p, 1.0f / 6.0f);
  p = fmaf(x, p, 0.5f);
  p = fmaf(x, p, 1.0f);
  const float small = x * p;
  const float large = __builtin_amdgcn_exp2f(x * 1.44269504088896341f) - 1.0f;
  return fabsf(x) <= 0.5f ? small : large;
}
// psi_s and reciprocals as a storage policy computes them: library expm1
// and IEEE division, or the cheaper forms for the 16-bit storages (kFast).
template <class St>
__device__ inline typename St::C psi_of(typename St::C rho, typename St::C rho0,
                                        typename St::C inv_rho0) {
  if constexpr (St::kFast) return -rho0 * expm1_fast(-rho * inv_rho0);
  else return psi_exp(rho, rho0, inv_rho0);
}
template <class St>
__device__ inline typename St::C recip(typename St::C v) {
  if constexpr (St::kFast) return __builtin_amdgcn_rcpf(v);  // 1 ulp
  else return typename St::C(1) / v;
}

template <unsigned kMode>
using Off = std::conditional_t<(kMode & kModeWide) != 0, uint64_t, uint32_t>;

// ---------------------------------------------------------------- memory
// Buffer resource word 3 for gfx9-family raw (untyped, unswizzled) access,
// and the cache-policy bit of a non-temporal store.
constexpr int kBufferWord3 = 0x00020000;
constexpr int kNonTemporal = 2;

// Population buffer access. Every byte offset is split into a uniform part
// `soff` (plane and row, held in a scalar register) and a per-lane part
// `voff` (column, plus a bounce-back displacement where a lane needs one).
// Below 4 GiB the buffer is accessed through a buffer resource, where the
// uniform part costs no vector instruction; the 64-bit variant adds both
// parts to a flat pointer.
template <class St, unsigned kMode>
struct PopMem {
  using T = typename St::T;
  using C = typename St::C;
  using O = Off<kMode>;
  using U2 = unsigned int __attribute__((ext_vector_type(2)));
  static constexpr bool kBuf = (kMode & kModeWide) == 0;
  __amdgpu_buffer_rsrc_t rsrc;
  char* base;
  __device__ PopMem(const void* p, uint64_t bytes) : base(static_cast<char*>(const_cast<void*>(p))) {
    if constexpr (kBuf)
      rsrc = __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)(uint32_t)bytes, kBufferWord3);
  }
  // FP32 rest planes of the kRest32 storages (byte offsets as for ld/st).
  __device__ float ldr(O soff, O voff) const {
    if constexpr (kBuf)
      return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, voff, soff, 0));
    else
      return *reinterpret_cast<const float*>(base + soff + voff);
  }
  __device__ void str(O soff, O voff, float v) const {
    if constexpr (kBuf)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), rsrc, voff, soff,
                                            kNonTemporal);
    else
      __builtin_nontemporal_store(v, reinterpret_cast<float*>(base + soff + voff));
  }
  __device__ C ld(O soff, O voff) const {
    if constexpr (kBuf) {
      if constexpr (sizeof(T) == 8)
        return St::decode(__builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff, soff, 0)));
      else if constexpr (sizeof(T) == 4)
        return St::decode(__builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rsrc, voff, soff, 0)));
      else
        return St::decode(__builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(rsrc, voff, soff, 0)));
    } else {
      return St::decode(*reinterpret_cast<const T*>(base + soff + voff));
    }
  }
  __device__ void st(O soff, O voff, C v) const {
    const T raw = St::encode(v);
    if constexpr (kBuf) {
      if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, raw), rsrc, voff, soff, kNonTemporal);
      else if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, raw), rsrc, voff, soff,
                                              kNonTemporal);
      else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, raw), rsrc, voff, soff,
                                              kNonTemporal);
    } else {
      __builtin_nontemporal_store(raw, reinterpret_cast<T*>(base + soff + voff));
    }
  }
};

// Bytes of a population buffer in units of one stored plane: 27 planes, and
// for kRest32 three FP32 rest planes of twice the size after them.
template <class St>
constexpr int kPlaneUnits = St::kRest32 ? 27 + 3 * (4 / (int)sizeof(typename St::T)) : 27;

// Per-lane byte offsets of one column x within a row (x itself and its
// periodic neighbours x - 1 and x + 1) and the uniform plane and row sizes;
// v0r is the column's offset in an FP32 rest plane (kRest32).
template <unsigned kMode>
struct LaneOff {
  Off<kMode> v0, vm, vp, v0r;
  Off<kMode> plane_b, row_b;
};

template <class St, unsigned kMode>
__device__ inline LaneOff<kMode> lane_off(int x, int lx, Off<kMode> plane_b, Off<kMode> row_b) {
  using O = Off<kMode>;
  constexpr int E = sizeof(typename St::T);
  LaneOff<kMode> L;
  L.v0 = (O)x * E;
  L.vm = (O)(x == 0 ? lx - 1 : x - 1) * E;
  L.vp = (O)(x == lx - 1 ? 0 : x + 1) * E;
  L.v0r = (O)x * 4;
  L.plane_b = plane_b;
  L.row_b = row_b;
  return L;
}

// Uniform byte offset of row r of the FP32 rest plane of set k (0 f_A,
// 1 f_B, 2 g) for the kRest32 storages: after the 27 16-bit planes, each
// rest plane and row twice the size of a 16-bit one.
template <class St, unsigned kMode>
__device__ inline Off<kMode> rest_off(const LaneOff<kMode>& L, int k, int r) {
  using O = Off<kMode>;
  constexpr O kRatio = 4 / sizeof(typename St::T);
  return (O)27 * L.plane_b + (O)k * kRatio * L.plane_b + (O)r * kRatio * L.row_b;
}

// Offsets of the value pulled for direction I into row r, in the block of
// nine planes that starts at byte `first`: plane I at row r - c_y, column
// x - c_x; or, where the link is solid (bounce-back), plane opp(I) at the
// node itself. The two alternatives differ by two planes and |c_y| rows;
// the uniform part is the lower of the two, so every lane offset is
// non-negative and a lane picks its alternative with its own offset alone.
template <unsigned kMode>
struct PullOff {
  Off<kMode> s, v;
};

// v + s evaluated where it is used: the displaced offsets of the rare
// bounce-back path are not hoisted out of the row loop, so they occupy no
// registers across it.
template <typename O>
__device__ inline O add_in_place(O v, O s) {
  if constexpr (sizeof(O) == 4) {
    O out;
    asm volatile("v_add_u32 %0, %1, %2" : "=v"(out) : "s"(s), "v"(v));
    return out;
  } else {
    return v + s;
  }
}

template <int I, unsigned kMode, bool kBounce>
__device__ inline PullOff<kMode> pull_off(const LaneOff<kMode>& L, Off<kMode> first, int r,
                                          bool bounce) {
  using O = Off<kMode>;
  constexpr int cx = Dir<I>::cx, cy = Dir<I>::cy, opp = Dir<I>::opp;
  const O shifted = cx > 0 ? L.vm : (cx < 0 ? L.vp : L.v0);
  PullOff<kMode> o;
  if constexpr (I == 0) {
    o.s = first + (O)r * L.row_b;
    o.v = L.v0;
  } else if constexpr (!kBounce) {
    o.s = first + (O)I * L.plane_b + (O)(r - cy) * L.row_b;
    o.v = shifted;
  } else {
    const O d = (O)2 * L.plane_b + (cy != 0 ? L.row_b : (O)0);
    if constexpr (opp > I) {
      o.s = first + (O)I * L.plane_b + (O)(r - cy) * L.row_b;
      o.v = bounce ? add_in_place(L.v0, d) : shifted;
    } else {
      o.s = first + (O)opp * L.plane_b + (O)r * L.row_b;
      o.v = bounce ? L.v0 : add_in_place(shifted, d);
    }
  }
  return o;
}

// Link-mask bits of the eight moving directions.
constexpr uint32_t kLinkBits = 0x1FEu;

// Whether any lane of the wavefront has a bounce-back link (uniform).
template <unsigned kMode>
__device__ inline bool any_link(uint32_t lm) {
  if constexpr ((kMode & kModeSolid) != 0) return __any((lm & kLinkBits) != 0u);
  else return (lm & kLinkBits) != 0u;  // flat walls: the mask depends on the row only
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
  const C tb = a.t_bottom[sx];  // loaded first: a select of values, not of addresses
  if (sr < 0) return tb;
  if (sr >= a.ly) return a.t_top;
  if constexpr ((kMode & kModeSolid) != 0) {
    const bool held_bottom = a.solid[(uint32_t)sr * (uint32_t)lx + (uint32_t)sx] == 1;
    return held_bottom ? tb : a.t_top;
  }
  return a.t_top;
}

// Momentum term of moving flat walls (the Couette walls of Sec. 2.2): a
// population bounced back at a wall that moves with u_w along x gains
// 6 w_i rho_w c_ix u_w, rho_w the node's own density at the previous time
// level (the sum of its post-collision populations). Only the diagonal links
// carry it (c_ix = 0 on the straight one), and the two diagonals of a wall
// cancel, so mass is conserved. Row 0 sees the bottom wall, row ly - 1 the
// top one; solid cells inside the lattice do not move.
template <class St, unsigned kMode, typename C>
__device__ inline void moving_wall_fluid(const StepArgs<C>& a, const PopMem<St, kMode>& m,
                                         const LaneOff<kMode>& L, int r, C (&f)[18]) {
  using O = Off<kMode>;
  const O p9 = L.plane_b * 9;
  C ra = 0, rb = 0;
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const O s = (O)j * L.plane_b + (O)r * L.row_b;
    if (St::kRest32 && j == 0) {
      ra += m.ldr(rest_off<St>(L, 0, r), L.v0r);
      rb += m.ldr(rest_off<St>(L, 1, r), L.v0r);
    } else {
      ra += m.ld(s, L.v0);
      rb += m.ld(s + p9, L.v0);
    }
  }
  if constexpr (St::kDev) {
    ra += a.ref_a;
    rb += a.ref_b;
  }
  if (r == 0) {  // links 5 (c_x = +1) and 6 (c_x = -1) come from the bottom wall
    const C k = C(6) * w_dir<C>(5) * a.uw0;
    f[5] = St::grid(f[5] + k * ra);
    f[14] = St::grid(f[14] + k * rb);
    f[6] = St::grid(f[6] - k * ra);
    f[15] = St::grid(f[15] - k * rb);
  }
  if (r == a.ly - 1) {  // links 8 (c_x = +1) and 7 (c_x = -1) from the top wall
    const C k = C(6) * w_dir<C>(8) * a.uw1;
    f[8] = St::grid(f[8] + k * ra);
    f[17] = St::grid(f[17] + k * rb);
    f[7] = St::grid(f[7] - k * ra);
    f[16] = St::grid(f[16] - k * rb);
  }
}

// Factor of the wall temperature in the anti-bounce-back of direction I at
// row r: the even part of the equilibrium at the wall velocity,
// 1 + 4.5 (c_I.u_w)^2 - 1.5 u_w^2, for a link whose source is a moving flat
// wall; 1 otherwise.
template <int I, unsigned kMode, typename C>
__device__ inline C wall_even_factor(const StepArgs<C>& a, int r) {
  if constexpr ((kMode & kModeMoving) == 0) {
    return C(1);
  } else {
    constexpr int cx = Dir<I>::cx, cy = Dir<I>::cy;
    const int sr = r - cy;
    if (sr >= 0 && sr < a.ly) return C(1);
    const C u = sr < 0 ? a.uw0 : a.uw1;
    return C(1) + (C(4.5) * C(cx * cx) - C(1.5)) * u * u;
  }
}

// Pull f_A (f[0..8]) and f_B (f[9..17]) of row r at lane column L, in
// stored form. Opposite directions have equal weights, so a bounced value
// keeps its deviation reference.
template <class St, unsigned kMode, typename C>
__device__ inline void pull_fluid(const StepArgs<C>& a, const PopMem<St, kMode>& m,
                                  const LaneOff<kMode>& L, int r, uint32_t lm, C (&f)[18]) {
  using O = Off<kMode>;
  const O p9 = L.plane_b * 9;
  if constexpr ((kMode & kModeInit) != 0) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const O s = (O)i * L.plane_b + (O)r * L.row_b;
      if (St::kRest32 && i == 0) {
        f[0] = m.ldr(rest_off<St>(L, 0, r), L.v0r);
        f[9] = m.ldr(rest_off<St>(L, 1, r), L.v0r);
      } else {
        f[i] = m.ld(s, L.v0);
        f[i + 9] = m.ld(s + p9, L.v0);
      }
    }
    return;
  }
#define TLB_PULL_F(I, B)                                                       \
  {                                                                            \
    const auto o = pull_off<I, kMode, B>(L, O(0), r, ((lm >> I) & 1u) != 0u);  \
    f[I] = m.ld(o.s, o.v);                                                     \
    f[I + 9] = m.ld(o.s + p9, o.v);                                            \
  }
  // the rest populations never move or bounce
  if constexpr (St::kRest32) {
    f[0] = m.ldr(rest_off<St>(L, 0, r), L.v0r);
    f[9] = m.ldr(rest_off<St>(L, 1, r), L.v0r);
  } else {
    TLB_PULL_F(0, false)
  }
  if (any_link<kMode>(lm)) {
    TLB_PULL_F(1, true) TLB_PULL_F(2, true) TLB_PULL_F(3, true)
    TLB_PULL_F(4, true) TLB_PULL_F(5, true) TLB_PULL_F(6, true) TLB_PULL_F(7, true)
    TLB_PULL_F(8, true)
    if constexpr ((kMode & kModeMoving) != 0) {
      if (r == 0 || r == a.ly - 1) moving_wall_fluid(a, m, L, r, f);
    }
  } else {
    TLB_PULL_F(1, false) TLB_PULL_F(2, false) TLB_PULL_F(3, false)
    TLB_PULL_F(4, false) TLB_PULL_F(5, false) TLB_PULL_F(6, false) TLB_PULL_F(7, false)
    TLB_PULL_F(8, false)
  }
#undef TLB_PULL_F
}

// Pull g of row r at lane column L (column index x), in stored form, with
// anti-bounce-back at solid sources: g_i = -g*_{opp i}(x) + 2 w_i T_w, i.e.
// in deviations from w_i T_ref: d_i = -d*_{opp i} + 2 w_i (T_w - T_ref).
template <class St, unsigned kMode, typename C>
__device__ inline void pull_thermal(const StepArgs<C>& a, const PopMem<St, kMode>& m,
                                    const LaneOff<kMode>& L, int x, int r, uint32_t lm,
                                    C (&g)[9]) {
  using O = Off<kMode>;
  const O p18 = L.plane_b * 18;
  if constexpr ((kMode & kModeInit) != 0) {
#pragma unroll
    for (int i = 0; i < 9; ++i)
      g[i] = (St::kRest32 && i == 0) ? m.ldr(rest_off<St>(L, 2, r), L.v0r)
                                     : m.ld(p18 + (O)i * L.plane_b + (O)r * L.row_b, L.v0);
    return;
  }
#define TLB_PULL_G(I, B)                                                          \
  {                                                                               \
    const bool bb = ((lm >> I) & 1u) != 0u;                                       \
    const auto o = pull_off<I, kMode, B>(L, p18, r, bb);                          \
    C v = m.ld(o.s, o.v);                                                         \
    if constexpr (B && I != 0) {                                                  \
      if (bb) {                                                                   \
        C tw = source_wall_temperature<I, kMode>(a, x, r) * wall_even_factor<I, kMode>(a, r); \
        if constexpr (St::kDev) tw -= a.ref_t;                                    \
        v = St::grid(C(2) * w_dir<C>(I) * tw - v);                                \
      }                                                                           \
    }                                                                             \
    g[I] = v;                                                                     \
  }
  if constexpr (St::kRest32) {
    g[0] = m.ldr(rest_off<St>(L, 2, r), L.v0r);
  } else {
    TLB_PULL_G(0, false)
  }
  if (any_link<kMode>(lm)) {
    TLB_PULL_G(1, true) TLB_PULL_G(2, true) TLB_PULL_G(3, true)
    TLB_PULL_G(4, true) TLB_PULL_G(5, true) TLB_PULL_G(6, true) TLB_PULL_G(7, true)
    TLB_PULL_G(8, true)
  } else {
    TLB_PULL_G(1, false) TLB_PULL_G(2, false) TLB_PULL_G(3, false)
    TLB_PULL_G(4, false) TLB_PULL_G(5, false) TLB_PULL_G(6, false) TLB_PULL_G(7, false)
    TLB_PULL_G(8, false)
  }
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
  const C tb = a.t_bottom[x];
  return a.solid[(uint32_t)y * (uint32_t)a.lx + (uint32_t)x] == 1 ? tb : a.t_top;
}

// ---------------------------------------------------------------- kernel
template <class St, int BX, unsigned kMode>
__global__ __launch_bounds__(BX) void lb_step_kernel(StepArgs<typename St::C> a) {
  using C = typename St::C;
  using T = typename St::T;
  using O = Off<kMode>;
  constexpr bool kTauOne = (kMode & kModeTauOne) != 0;
  constexpr int kKept = kTauOne ? 4 : 18;  // values kept per pulled row
  constexpr int W = BX + 4;   // ring row width: strip plus 2 halo columns each side
  constexpr int R = 6;        // ring rows
  __shared__ C s_rho[2][R][W];
  __shared__ C s_psi[2][R][W];

  const int lx = a.lx, ly = a.ly;
  const int tid = threadIdx.x;
  // Tile order. Workgroups are dispatched to the eight XCDs round-robin by
  // linear id, and each XCD has its own L2; the linear id is remapped so
  // that each XCD receives a contiguous run of tiles (strip fastest), and
  // tiles that share halo columns run on the same L2 at the same time.
  // Odd row chunks march downwards, so two neighbouring chunks reach their
  // shared halo rows at the same time (both at the start or both at the end).
  const int nbx = gridDim.x;
  const int ntiles = gridDim.x * gridDim.y;
  const int lin = blockIdx.y * nbx + blockIdx.x;
  constexpr int kXcds = 8;
  const int xcd = lin % kXcds;
  const int tile = xcd * (ntiles / kXcds) + min(xcd, ntiles % kXcds) + lin / kXcds;
  const int chunk = tile / nbx;
  const int x0 = (tile - chunk * nbx) * BX;
  const int y0 = chunk * a.rows_per_block;
  const int y1 = min(y0 + a.rows_per_block, ly);
  const bool down = (chunk & 1) != 0;
  const O row_b = (O)a.pitch * sizeof(T);
  const O plane_b = (O)a.pop_stride * sizeof(T);
  const PopMem<St, kMode> msrc(a.src, (uint64_t)plane_b * kPlaneUnits<St>);
  const PopMem<St, kMode> mdst(a.dst, (uint64_t)plane_b * kPlaneUnits<St>);

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
  const LaneOff<kMode> Lo = lane_off<St, kMode>(xw, lx, plane_b, row_b);
  const LaneOff<kMode> Lh = lane_off<St, kMode>(hx, lx, plane_b, row_b);

  const C psi_w0 = psi_of<St>(a.rho_wall0, a.rho0, a.inv_rho0);
  const C psi_w1 = psi_of<St>(a.rho_wall1, a.rho0, a.inv_rho0);

  double acc[kObsSums] = {0, 0, 0, 0, 0, 0};

  // Link mask of node (x, r), solid outside the lattice. With solid cells it
  // is a global load, issued one row iteration before the row is pulled so
  // that its latency does not delay the population loads that depend on it.
  auto mask_at = [&](int x, int r) -> uint32_t {
    return (r >= 0 && r < ly) ? link_mask<kMode>(a, x, r) : kSelfSolid;
  };

  // Densities of node (x, r) with link mask lm_in into ring slot `slot` /
  // column `col`; the pulled populations land in f and the mask in lm.
  // Returns whether the node was pulled (fluid, inside the lattice).
  auto density = [&](const LaneOff<kMode>& L, int r, uint32_t lm_in, int slot, int col,
                     C (&f)[18], uint32_t& lm) {
    C ra = a.rho_wall0, rb = a.rho_wall1, pa = psi_w0, pb = psi_w1;
    bool pulled = false;
    lm = kSelfSolid;
    if (r >= 0 && r < ly) {
      lm = lm_in;
      if (!((kMode & kModeSolid) != 0 && (lm & kSelfSolid))) {
        pull_fluid<St, kMode>(a, msrc, L, r, lm, f);
        ra = sum9(f);
        rb = sum9(f + 9);
        if constexpr (St::kDev) {
          ra += a.ref_a;
          rb += a.ref_b;
        }
        pa = psi_of<St>(ra, a.rho0, a.inv_rho0);
        pb = psi_of<St>(rb, a.rho0, a.inv_rho0);
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
  const int dir = down ? -1 : 1;
  const int r_first = down ? y1 + 1 : y0 - 2;
  // prefetched masks of the next pulled row: own column, and the halo
  // column of lanes 0..3 (each wavefront keeps its own, used in its turn)
  uint32_t pm_own = mask_at(xw, r_first), pm_halo = lane < 4 ? mask_at(hx, r_first) : kSelfSolid;
  auto iterate = [&](int k, C (&kw)[kKept], uint32_t& lw, const C (&ku)[kKept], uint32_t lu) {
    const int r = r_first + dir * k;
    const int y = down ? r + 2 : r - 2;
    const uint32_t m_own = pm_own, m_halo = pm_halo;
    pm_own = mask_at(xw, r + dir);
    if (lane < 4) pm_halo = mask_at(hx, r + dir);
    const int slot = k % R;
    const bool out = k >= 4 && y >= y0 && y < y1 && own_valid;
    const bool out_fluid = out && !((kMode & kModeSolid) != 0 && (lu & kSelfSolid));
    const O yrow = (O)(y < 0 ? 0 : y) * row_b;
    C g[9];
    if (out_fluid) pull_thermal<St, kMode>(a, msrc, Lo, xw, y, lu, g);
    {
      C f[18];
      const bool pulled = density(Lo, r, m_own, slot, tid + 2, f, lw);
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
      density(Lh, r, m_halo, slot, hslot, hf, hl);
    }
    __syncthreads();

    if (!out) return;
    if (!out_fluid) {
      if constexpr ((kMode & kModeStore) != 0) {
#pragma unroll
        for (int p = 0; p < 27; ++p) {
          if (St::kRest32 && p % 9 == 0) mdst.str(rest_off<St>(Lo, p / 9, y < 0 ? 0 : y), Lo.v0r, 0.0f);
          else mdst.st((O)p * plane_b + yrow, Lo.v0, C(0));
        }
      }
      if constexpr ((kMode & kModeFields) != 0) {
        const size_t nn = (size_t)lx * ly, q = (size_t)y * lx + xo;
        a.fields[q] = (double)a.rho_wall0;
        a.fields[nn + q] = (double)a.rho_wall1;
        a.fields[2 * nn + q] = 0.0;
        a.fields[3 * nn + q] = 0.0;
        a.fields[4 * nn + q] = (double)solid_temperature(a, xo, y);
        if constexpr ((kMode & kModeStress) != 0) {
          a.fields[5 * nn + q] = 0.0;
          a.fields[6 * nn + q] = 0.0;
        }
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
    for (int d = 0; d < 5; ++d) rs[d] = (down ? k + 6 - d : k + 2 + d) % R;  // d = dy + 2
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
    const C inv_rho = recip<St>(rho);
    const C ux = jx * inv_rho, uy = jy * inv_rho;
    const C Fx = FA[0] + FB[0], Fy = FA[1] + FB[1];
    const C hx = ux + C(0.5) * Fx * inv_rho;
    const C hy = uy + C(0.5) * Fy * inv_rho;

    if constexpr ((kMode & kModeStore) != 0) {
      const C tA = a.tau * recip<St>(ra), tB = a.tau * recip<St>(rb);
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
    // Opposite directions share the even part of the equilibrium:
    // f^eq_{i, opp i} = S_i +- D_i with S_i = w_i rho (1 + 4.5 (c_i.u)^2
    // - 1.5 u^2) and D_i = 3 w_i rho (c_i.u), so each pair costs one S and
    // one D per field.
#define TLB_PAIR(I)                                                                    \
  {                                                                                    \
    constexpr int J = Dir<I>::opp;                                                     \
    constexpr int cx = Dir<I>::cx, cy = Dir<I>::cy;                                   \
    constexpr C w = w_dir<C>(I);                                                       \
    const C cua = C(cx) * uax + C(cy) * uay;                                           \
    const C cub = C(cx) * ubx + C(cy) * uby;                                           \
    const C cuh = C(cx) * hx + C(cy) * hy;                                             \
    C Sa = w * ra * (C(1) + C(4.5) * cua * cua - C(1.5) * ua2);                        \
    C Sb = w * rb * (C(1) + C(4.5) * cub * cub - C(1.5) * ub2);                        \
    C Sg = w * temp * (C(1) + C(4.5) * cuh * cuh - C(1.5) * uh2);                      \
    const C Dla = C(3) * w * ra * cua;                                                 \
    const C Dlb = C(3) * w * rb * cub;                                                 \
    const C Dlg = C(3) * w * temp * cuh;                                               \
    if constexpr (St::kDev) {                                                          \
      Sa -= w * a.ref_a;                                                               \
      Sb -= w * a.ref_b;                                                               \
      Sg -= w * a.ref_t;                                                               \
    }                                                                                  \
    const C eaI = Sa + Dla, eaJ = Sa - Dla;                                            \
    const C ebI = Sb + Dlb, ebJ = Sb - Dlb;                                            \
    const C egI = Sg + Dlg, egJ = Sg - Dlg;                                            \
    C qaI = eaI, qaJ = eaJ, qbI = ebI, qbJ = ebJ, qgI = egI, qgJ = egJ;               \
    if constexpr (!kTauOne) {                                                          \
      qaI += ka * (fa[I] - eaI);                                                       \
      qaJ += ka * (fa[J] - eaJ);                                                       \
      qbI += ka * (fb[I] - ebI);                                                       \
      qbJ += ka * (fb[J] - ebJ);                                                       \
      qgI += kg * (g[I] - egI);                                                        \
      qgJ += kg * (g[J] - egJ);                                                        \
    }                                                                                  \
    qaI = St::stored(qaI);                                                             \
    qaJ = St::stored(qaJ);                                                             \
    qbI = St::stored(qbI);                                                             \
    qbJ = St::stored(qbJ);                                                             \
    qgI = St::stored(qgI);                                                             \
    qgJ = St::stored(qgJ);                                                             \
    if constexpr (St::kFix || St::kRest32) {                                           \
      sa += qaI + qaJ;                                                                 \
      sb += qbI + qbJ;                                                                 \
      sg += qgI + qgJ;                                                                 \
    } else {                                                                           \
      sa += eaI + eaJ;                                                                 \
      sb += ebI + ebJ;                                                                 \
      sg += egI + egJ;                                                                 \
    }                                                                                  \
    const O oI = (O)I * plane_b + yrow, oJ = (O)J * plane_b + yrow;                    \
    mdst.st(oI, Lo.v0, qaI);                                                           \
    mdst.st(oJ, Lo.v0, qaJ);                                                           \
    mdst.st(oI + p9, Lo.v0, qbI);                                                      \
    mdst.st(oJ + p9, Lo.v0, qbJ);                                                      \
    mdst.st(oI + p18, Lo.v0, qgI);                                                     \
    mdst.st(oJ + p18, Lo.v0, qgJ);                                                     \
  }
      TLB_PAIR(1) TLB_PAIR(2) TLB_PAIR(5) TLB_PAIR(6)
#undef TLB_PAIR
      if constexpr (St::kFix) {
        // exact remainders: the stored populations sum to the pulled ones
        mdst.st(yrow, Lo.v0, St::grid(Da - sa));
        mdst.st(yrow + p9, Lo.v0, St::grid(Db - sb));
        mdst.st(yrow + p18, Lo.v0, St::grid(Dt - sg));
      } else if constexpr (St::kRest32) {
        // FP32 remainders of the rounded moving populations (any tau: the
        // BGK rest value is the zeroth moment minus the other eight)
        mdst.str(rest_off<St>(Lo, 0, y), Lo.v0r, Da - sa);
        mdst.str(rest_off<St>(Lo, 1, y), Lo.v0r, Db - sb);
        mdst.str(rest_off<St>(Lo, 2, y), Lo.v0r, Dt - sg);
      } else if constexpr (kTauOne) {
        mdst.st(yrow, Lo.v0, Da - sa);
        mdst.st(yrow + p9, Lo.v0, Db - sb);
        mdst.st(yrow + p18, Lo.v0, Dt - sg);
      } else {
        const C ea = Da - sa, eb = Db - sb, eg = Dt - sg;
        mdst.st(yrow, Lo.v0, ea + ka * (fa[0] - ea));
        mdst.st(yrow + p9, Lo.v0, eb + ka * (fb[0] - eb));
        mdst.st(yrow + p18, Lo.v0, eg + kg * (g[0] - eg));
      }
    }
    if constexpr ((kMode & kModeMoments) != 0) {
      static_assert(!St::kDev && !St::kFix, "moments of the FP64 / FP32 storages");
      C* mo = static_cast<C*>(a.moments);
      const size_t ps = (size_t)a.pop_stride, q = (size_t)y * (size_t)a.pitch + (size_t)xo;
      mo[q] = ra;
      mo[ps + q] = rb;
      mo[2 * ps + q] = jx;
      mo[3 * ps + q] = jy;
      mo[4 * ps + q] = temp;
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
      if constexpr ((kMode & kModeStress) != 0) {
        static_assert(!kTauOne, "the stress needs the pulled populations");
        // viscous part: -(1 - 1/(2 tau)) sum_l sum_i c_ix c_iy (f_{l,i} -
        // f^eq_i(rho_l, u_l)); the deviation references carry no xy moment
        const C tA = a.tau * recip<St>(ra), tB = a.tau * recip<St>(rb);
        const C uax = ux + FA[0] * tA, uay = uy + FA[1] * tA;
        const C ubx = ux + FB[0] * tB, uby = uy + FB[1] * tB;
        const C pia = (fa[5] + fa[7]) - (fa[6] + fa[8]);
        const C pib = (fb[5] + fb[7]) - (fb[6] + fb[8]);
        const C visc = -(C(1) - C(0.5) * a.inv_tau) * ((pia - ra * uax * uay) + (pib - rb * ubx * uby));
        // interaction pressure tensor: 1/2 sum_l psi_l(x) sum_c G(c) psi_l(x+c)
        // c_x c_y (self) and 1/2 G12 sum_l psi_x,l(x) sum_c w(c) psi_x,m(x+c)
        // c_x c_y (cross); c and -c share c_x c_y, so each pair is one term
        C pint = 0;
#pragma unroll
        for (int l = 0; l < 2; ++l) {
          const C ga = l == 0 ? a.ga0 : a.ga1;
          const C gr = l == 0 ? a.gr0 : a.gr1;
          C self = 0;
#pragma unroll
          for (int dx = 1; dx <= 2; ++dx) {
#pragma unroll
            for (int dy = -2; dy <= 2; ++dy) {
              if (dy == 0) continue;
              const int c2 = dx * dx + dy * dy;
              const C gw = ga * w_c2<C>(c2) + gr * p_c2<C>(c2);
              self += gw * C(dx * dy) *
                      (s_psi[l][rs[dy + 2]][s0 + dx] + s_psi[l][rs[2 - dy]][s0 - dx]);
            }
          }
          const int m = 1 - l;
          C cross = 0;
#pragma unroll
          for (int dy = -1; dy <= 1; dy += 2)
            cross += w_c2<C>(2) * C(dy) *
                     (s_rho[m][rs[dy + 2]][s0 + 1] + s_rho[m][rs[2 - dy]][s0 - 1]);
          const C rl = l == 0 ? ra : rb;
          pint += C(0.5) * s_psi[l][rs[2]][s0] * self +
                  C(0.5) * a.g12 * a.inv_rho0 * a.inv_rho0 * rl * cross;
        }
        a.fields[5 * nn + q] = (double)visc;
        a.fields[6 * nn + q] = (double)pint;
      }
    }
    if constexpr ((kMode & kModeObserve) != 0) {
      // local sums only: the fluid-node sum of the central differences of T
      // (Nu's conductive term) telescopes along each column to the wall
      // temperatures and is formed on the host
      acc[0] += dra;
      acc[1] += drb;
      acc[2] += dtt;
      acc[3] += (double)hy * dtt;
      acc[4] += (double)hx * (double)hx + (double)hy * (double)hy;
      if (y == ly - 1) acc[5] += dtt - (double)a.t_top;
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
    // block reduction of the sums in a fixed order (deterministic)
    __shared__ double s_acc[BX / 64][kObsSums];
#pragma unroll
    for (int j = 0; j < kObsSums; ++j) {
      double v = acc[j];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
      if ((tid & 63) == 0) s_acc[tid >> 6][j] = v;
    }
    __syncthreads();
    if (tid < kObsSums) {
      double v = 0;
      for (int w = 0; w < BX / 64; ++w) v += s_acc[w][tid];
      a.partials[(size_t)lin * kObsSums + tid] = v;
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
      const C d = St::stored(v - w_dir<C>(i) * ref[s]);   // stored form
      sum[s] += (St::kFix || St::kRest32) ? d : v;
      St::store(buf + (long long)(i + 9 * s) * pop_stride + off, is_solid ? C(0) : d);
    }
  }
  // rest population: zeroth moment minus the other eight (exact mass)
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    if constexpr (St::kRest32) {
      float* rest = reinterpret_cast<float*>(buf + 27 * pop_stride) + (long long)s * pop_stride;
      __builtin_nontemporal_store(is_solid ? 0.0f : (dens[s] - ref[s]) - sum[s], rest + off);
    } else {
      const C d = St::kFix ? St::grid(St::grid(dens[s] - ref[s]) - sum[s])
                           : (dens[s] - sum[s]) - w_dir<C>(0) * ref[s];
      St::store(buf + (long long)(9 * s) * pop_stride + off, is_solid ? C(0) : d);
    }
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
  const long long off = (long long)y * pitch + x;
  double v;
  if (St::kRest32 && p % 9 == 0)
    v = (double)(reinterpret_cast<const float*>(buf + 27 * pop_stride) + (long long)(p / 9) * pop_stride)[off];
  else
    v = (double)St::load(buf + p * pop_stride + off);
  if constexpr (St::kDev)
    v += w_dir<double>(p % 9) * (double)(p < 9 ? ref_a : (p < 18 ? ref_b : ref_t));
  if (solid[(size_t)y * lx + x] != 0) v = 0.0;
  out[((size_t)p * ly + y) * lx + x] = v;
}

}  // namespace tlbk
