// Fused two-step update f*(t) -> f*(t+2) for tau = tau_g = 1 (arXiv:2109.12565,
// Sec. 2): FP64, FP32 and the 16-bit floating deviation storages (their
// intermediate level stays in FP32, so a fused launch rounds to 16 bits once
// per two steps), solid cells allowed, flat walls at rest or moving along x.
//
// At tau = tau_g = 1 the BGK collision (Eqs. (2), (16)) returns the
// equilibria (Eqs. (3), (18)), so the post-collision populations of a node
// are fixed by nine moments: rho_A and u_A, rho_B and u_B (the velocities
// shifted by the force, Eq. (6)), T and u^H. One launch therefore advances
// two time steps while the 27 population planes cross HBM once:
//
//   level 1  the ordinary step on the populations of time t read from HBM
//            (pull with half-way bounce-back and anti-bounce-back, Sec. 2.2;
//            moments; psi in an LDS ring; forces, Eqs. (7)-(11), (22);
//            velocities), ending in the moments of each node, which go to
//            an LDS ring instead of HBM: per field (f_A, f_B, g) its density
//            rho (or T), velocity u and u^2, one 16-byte vector each;
//   level 2  pulls each population of time t+1 from the moments of its
//            source node with the expressions the single step stores it
//            with (even part S and odd part D of the pair of directions),
//            the rest population as the remainder of the zeroth moment,
//            then completes the step and stores f*(t+2) with 27 aligned
//            stores.
//
// Two fused steps therefore give the numbers of two single steps up to the
// contraction of multiply-adds, which the compiler may choose differently in
// the two kernels. The pulled values and the ones subtracted for the rest
// population must round alike, though (see pull_level2).
//
// Halo. Level-2 collisions of a lane need level-2 densities of the lanes
// within 2, which need level-1 moments within 3, which need level-1
// densities within 5. A block of BT lanes computes BT consecutive (periodic)
// columns and stores the middle ones; neighbouring strips overlap by 10
// columns, so no lane does halo work of another kind. In y the chunk's rows
// are extended by 5 rows of level 1 on each side.
//
// Row pipeline. Iteration k handles four rows in two phases separated by
// barriers (up-marching chunk; a down-marching chunk mirrors the offsets):
//   phase 1  issue the HBM pulls of row ra (f) and of row rb = ra - 2 (g);
//            level-2 pull of row rc = ra - 4 from the moment ring into the
//            level-2 density ring (hiding the load latency); level-1
//            densities of row ra into the level-1 density ring;
//   phase 2  level-1 forces and moments of row rb into the moment ring;
//            level-2 forces, collision and stores of row rd = ra - 6.
// The density rings hold 5 rows and the moment ring 3 (rows by absolute
// index); each ring row written in one phase is read only after the next
// barrier and overwritten only after every read of it.
#pragma once

#include "lb_kernels.hpp"

namespace tlbk {

// Ring slot of row r for a ring of R rows (r >= -8 R).
template <int R>
__device__ inline int ring_slot(int r) {
  return (r + 8 * R) % R;
}

// Even and odd parts of the equilibrium of the direction pair P, opp(P):
// f^eq_P = S + D, f^eq_opp(P) = S - D (Eqs. (3), (18)); the same expressions
// as the single-step collision.
template <int P, typename C>
__device__ inline void eq_even_odd(C rho, C ux, C uy, C u2, C& S, C& D) {
  constexpr int cx = Dir<P>::cx, cy = Dir<P>::cy;
  constexpr C w = w_dir<C>(P);
  const C cu = C(cx) * ux + C(cy) * uy;
  S = w * rho * (C(1) + C(4.5) * cu * cu - C(1.5) * u2);
  D = C(3) * w * rho * cu;
}

// Forces on both components at ring column s0, rows rs[0..4] = dy -2..2:
// self interaction with nearest-neighbour attraction and 25-point repulsion
// (Eqs. (10), (11), weights of Fig. 1(b)), cross repulsion with
// psi = rho / rho0 (Eqs. (7), (8)), buoyancy (Eq. (22)). Same arithmetic as
// the single-step kernel.
template <typename C, int R, int W>
__device__ inline void step2_forces(const StepArgs<C>& a, const C (&s_rho)[2][R][W],
                                    const C (&s_psi)[2][R][W], const int (&rs)[5], int s0, C ra,
                                    C rb, C temp, C (&FA)[2], C (&FB)[2]) {
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    C ax = 0, ay = 0, qx = 0, qy = 0;
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
  FA[1] += ra * a.alpha_g * temp;
  FB[1] += rb * a.alpha_g * temp;
}

// Moments of a level-1 node for one field: the density (or temperature)
// rho, the velocity u and u2 = |u|^2; the moment ring holds three per node
// (f_A, f_B, g), read as 16-byte vectors.
template <typename C>
struct alignas(4 * sizeof(C)) Mom4 {
  C rho, ux, uy, u2;
};

// Sum of the eight moving equilibria of a node in the single step's order
// and form: ((S + D) + (S - D)) over the pairs 1, 2, 5, 6.
template <typename C>
__device__ inline C moving_sum(const Mom4<C>& m) {
  C sum = 0;
#define TLB_SUM_PAIR(P)                                 \
  {                                                     \
    C S, D;                                             \
    eq_even_odd<P>(m.rho, m.ux, m.uy, m.u2, S, D);      \
    sum += (S + D) + (S - D);                           \
  }
  TLB_SUM_PAIR(1) TLB_SUM_PAIR(2) TLB_SUM_PAIR(5) TLB_SUM_PAIR(6)
#undef TLB_SUM_PAIR
  return sum;
}

// Level-2 pull of direction I (1..8) at a node from the moment ring: the
// value f*_I(x - c_I) of the source node, or, across a solid link, the
// node's own f*_opp(I) (bounce-back) and 2 w_I T_w - g*_opp(I) (anti-
// bounce-back). Both alternatives belong to the pair of I, so a lane
// selects its ring cell and the sign of the odd part.
// kBounce = false: no lane of the wavefront has a solid link, so the ring
// cell and the sign are the same for every lane and known at compile time.
template <int I, bool kBounce, unsigned kMode, typename C, int RM, int WM>
__device__ inline void pull_level2(const StepArgs<C>& a, const Mom4<C> (&sm)[RM][WM][3],
                                   int slot_own, int col_own, int x, int r, uint32_t lm,
                                   C (&fa)[9], C (&fb)[9], C (&g)[9]) {
  // The odd part is added as in the rest population's sum and in the single
  // step's stores, without contracting it into a fused multiply-add: a pulled
  // value rounded differently from the one subtracted for the source's rest
  // population leaves a rounding mismatch that the interface dynamics amplify
  // (FP32 after 1000 steps: 8e-6 of rho against the oracle instead of 3e-6).
#pragma clang fp contract(off)
  constexpr int P = (I == 1 || I == 2 || I == 5 || I == 6) ? I : Dir<I>::opp;
  const bool bb = kBounce && ((lm >> I) & 1u) != 0u;
  const int s = bb ? slot_own : ring_slot<RM>(r - Dir<I>::cy);
  const int c = bb ? col_own : col_own - Dir<I>::cx;
  const Mom4<C>* src = sm[s][c];
  const Mom4<C> ma = src[0], mb = src[1], mg = src[2];
  C Sa, Da, Sb, Db, Sg, Dg;
  eq_even_odd<P>(ma.rho, ma.ux, ma.uy, ma.u2, Sa, Da);
  eq_even_odd<P>(mb.rho, mb.ux, mb.uy, mb.u2, Sb, Db);
  eq_even_odd<P>(mg.rho, mg.ux, mg.uy, mg.u2, Sg, Dg);
  const bool plus = (P == I) != bb;
  fa[I] = plus ? Sa + Da : Sa - Da;
  fb[I] = plus ? Sb + Db : Sb - Db;
  C v = plus ? Sg + Dg : Sg - Dg;
  if (bb) {
    const C tw = source_wall_temperature<I, kMode>(a, x, r) * wall_even_factor<I, kMode>(a, r);
    v = C(2) * w_dir<C>(I) * tw - v;
  }
  g[I] = v;
}

template <class St, int BT, unsigned kMode>
__global__ __launch_bounds__(BT) void lb_step2_kernel(StepArgs<typename St::C> a, int strip_w) {
  using C = typename St::C;
  using O = Off<kMode>;
  static_assert(!St::kFix && (!St::kDev || St::kRest32),
                "two-step kernel: FP64, FP32, or 16-bit floating deviations with FP32 rest planes");
  static_assert((kMode & kModeTauOne) != 0 && (kMode & kModeStore) != 0, "tau = 1 store pass");
  static_assert((kMode & (kModeWide | kModeInit | kModeObserve | kModeFields)) == 0,
                "32-bit offsets, no observables");
  constexpr bool kTop = (kMode & kModeTopRow) != 0;
  constexpr bool kMoments = (kMode & kModeMoments) != 0;
  static_assert(!kMoments || !St::kDev, "moments of the FP64 / FP32 storages");
  constexpr int kH = 5;          // left halo lanes
  constexpr int R1 = 5, RM = 3;  // density ring rows, moment ring rows
  constexpr int W = BT + 4;      // density ring row: lanes plus 2 padding columns each side
  constexpr int WM = BT + 2;     // moment ring row: 1 padding column each side
  __shared__ C s1_rho[2][R1][W];
  __shared__ C s1_psi[2][R1][W];
  __shared__ C s2_rho[2][R1][W];
  __shared__ C s2_psi[2][R1][W];
  __shared__ Mom4<C> sm[RM][WM][3];

  const int lx = a.lx, ly = a.ly;
  const int tid = threadIdx.x;
  // XCD-aware tile order and alternating chunk direction, as in the single
  // step (each XCD receives a contiguous run of tiles).
  const int nbx = gridDim.x;
  const int ntiles = gridDim.x * gridDim.y;
  const int lin = blockIdx.y * nbx + blockIdx.x;
  constexpr int kXcds = 8;
  const int xcd = lin % kXcds;
  const int tile = xcd * (ntiles / kXcds) + min(xcd, ntiles % kXcds) + lin / kXcds;
  const int chunk = tile / nbx;
  const int x0 = (tile - chunk * nbx) * strip_w;
  const int y0 = chunk * a.rows_per_block;
  const int y1 = min(y0 + a.rows_per_block, ly);
  const bool down = (chunk & 1) != 0;

  using T = typename St::T;
  const O row_b = (O)a.pitch * sizeof(T);
  const O plane_b = (O)a.pop_stride * sizeof(T);
  const PopMem<St, kMode> msrc(a.src, (uint64_t)plane_b * kPlaneUnits<St>);
  const PopMem<St, kMode> mdst(a.dst, (uint64_t)plane_b * kPlaneUnits<St>);

  // lane column (periodic); lanes kH .. kH + strip_w - 1 inside the lattice
  // store, the others compute halo columns only
  const int xl = x0 - kH + tid;
  const int xw = ((xl % lx) + lx) % lx;
  const bool out_lane = tid >= kH && tid < kH + strip_w && xl < lx;
  const LaneOff<kMode> Lo = lane_off<St, kMode>(xw, lx, plane_b, row_b);
  const int c1 = tid + 2;  // column in the density rings
  const int cm = tid + 1;  // column in the moment ring
  // kMoments: moments of the pulled state of each level, [level][5][pop_stride]
  auto put_moments = [&](int level, int r, C rho_a, C rho_b, C jx, C jy, C temp) {
    C* mo = static_cast<C*>(a.moments) + (size_t)level * 5 * (size_t)a.pop_stride;
    const size_t ps = (size_t)a.pop_stride, q = (size_t)r * (size_t)a.pitch + (size_t)xw;
    mo[q] = rho_a;
    mo[ps + q] = rho_b;
    mo[2 * ps + q] = jx;
    mo[3 * ps + q] = jy;
    mo[4 * ps + q] = temp;
  };

  const C psi_w0 = psi_of<St>(a.rho_wall0, a.rho0, a.inv_rho0);
  const C psi_w1 = psi_of<St>(a.rho_wall1, a.rho0, a.inv_rho0);
  constexpr bool kSolid = (kMode & kModeSolid) != 0;
  // kTop: this lane's T - t_top on the top row at the two levels (the chunk
  // that owns the top row, stored lanes only: each column counted once)
  const bool top_chunk = kTop && y1 == ly;
  double top_sum[2] = {0.0, 0.0};

  // Level 1, phase 1: pull row ra from HBM (issued first in the phase, so
  // the level-2 work of the phase hides the load latency), then densities
  // and psi into ring 1 and the kept rho_A, rho_B, j (tau = 1: the moments
  // are all the collision needs).
  // Link mask of row r at the lane's column (solid for rows outside the
  // lattice). With solid cells it is a global load, issued one row
  // iteration before the row is pulled so that its latency does not delay
  // the loads (level 1) or LDS reads (level 2) that depend on it.
  auto mask_of = [&](int r) -> uint32_t {
    return (r >= 0 && r < ly) ? link_mask<kMode>(a, xw, r) : kSelfSolid;
  };
  auto level1_pull = [&](int r, uint32_t lm, C (&f)[18], uint32_t& lw) {
    lw = lm;
    if (r >= 0 && r < ly && !(kSolid && (lw & kSelfSolid))) pull_fluid<St, kMode>(a, msrc, Lo, r, lw, f);
  };
  auto level1_density = [&](int r, const C (&f)[18], uint32_t lw, C (&kw)[4]) {
    C ra = a.rho_wall0, rb = a.rho_wall1, pa = psi_w0, pb = psi_w1;
    if (r >= 0 && r < ly && !(kSolid && (lw & kSelfSolid))) {
      // densities in full (the deviation storages add their references; the
      // references carry no momentum)
      kw[0] = sum9(f);
      kw[1] = sum9(f + 9);
      if constexpr (St::kDev) {
        kw[0] += a.ref_a;
        kw[1] += a.ref_b;
      }
      kw[2] = momentum_x(f, f + 9);
      kw[3] = momentum_y(f, f + 9);
      ra = kw[0];
      rb = kw[1];
      pa = psi_of<St>(ra, a.rho0, a.inv_rho0);
      pb = psi_of<St>(rb, a.rho0, a.inv_rho0);
    }
    const int s = ring_slot<R1>(r);
    s1_rho[0][s][c1] = ra;
    s1_rho[1][s][c1] = rb;
    s1_psi[0][s][c1] = pa;
    s1_psi[1][s][c1] = pb;
  };

  // Level 1, phase 2: forces and velocities of fluid row r; per field its
  // density (or temperature), velocity and u^2 into the moment ring.
  auto level1_moments = [&](int r, const C (&ku)[4], const C (&g)[9]) {
    const C Da = ku[0], Db = ku[1], jx = ku[2], jy = ku[3];
    const C ra = Da, rb = Db;
    C Dt = sum9(g);
    if constexpr (St::kDev) Dt += a.ref_t;
    const C temp = Dt;
    if constexpr (kTop) {
      if (top_chunk && r == ly - 1 && out_lane) top_sum[0] += (double)temp - (double)a.t_top;
    }
    int rs[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) rs[d] = ring_slot<R1>(r - 2 + d);
    C FA[2], FB[2];
    step2_forces(a, s1_rho, s1_psi, rs, c1, ra, rb, temp, FA, FB);
    const C rho = ra + rb;
    const C inv_rho = recip<St>(rho);
    const C ux = jx * inv_rho, uy = jy * inv_rho;
    const C Fx = FA[0] + FB[0], Fy = FA[1] + FB[1];
    const C hx = ux + C(0.5) * Fx * inv_rho;
    const C hy = uy + C(0.5) * Fy * inv_rho;
    const C tA = a.tau * recip<St>(ra), tB = a.tau * recip<St>(rb);
    const C uax = ux + FA[0] * tA, uay = uy + FA[1] * tA;
    const C ubx = ux + FB[0] * tB, uby = uy + FB[1] * tB;
    const C ua2 = uax * uax + uay * uay;
    const C ub2 = ubx * ubx + uby * uby;
    const C uh2 = hx * hx + hy * hy;
    Mom4<C>* m = sm[ring_slot<RM>(r)][cm];
    const Mom4<C> mv[3] = {{Da, uax, uay, ua2}, {Db, ubx, uby, ub2}, {Dt, hx, hy, uh2}};
    m[0] = mv[0];
    m[1] = mv[1];
    m[2] = mv[2];
    if constexpr (kMoments) {
      if (out_lane && r >= y0 && r < y1) put_moments(0, r, Da, Db, jx, jy, Dt);
    }
  };

  // Level 2, phase 1: pull row r from the moment ring; densities and psi
  // into ring 2; keep rho_A, rho_B, j, T.
  auto level2_density = [&](int r, uint32_t lm, C (&kw)[5], uint32_t& lw) {
    C ra = a.rho_wall0, rb = a.rho_wall1, pa = psi_w0, pb = psi_w1;
    lw = lm;
    if (r >= 0 && r < ly) {
      if (!(kSolid && (lw & kSelfSolid))) {
        const int so = ring_slot<RM>(r);
        C fa[9], fb[9], g[9];
        {
          // rest populations: the zeroth moments minus the moving
          // equilibria, as the single step stores them
          const Mom4<C>* m = sm[so][cm];
          fa[0] = m[0].rho - moving_sum(m[0]);
          fb[0] = m[1].rho - moving_sum(m[1]);
          g[0] = m[2].rho - moving_sum(m[2]);
        }
#define TLB_PULL2(B)                                                   \
  pull_level2<1, B, kMode>(a, sm, so, cm, xw, r, lw, fa, fb, g);       \
  pull_level2<2, B, kMode>(a, sm, so, cm, xw, r, lw, fa, fb, g);       \
  pull_level2<3, B, kMode>(a, sm, so, cm, xw, r, lw, fa, fb, g);       \
  pull_level2<4, B, kMode>(a, sm, so, cm, xw, r, lw, fa, fb, g);       \
  pull_level2<5, B, kMode>(a, sm, so, cm, xw, r, lw, fa, fb, g);       \
  pull_level2<6, B, kMode>(a, sm, so, cm, xw, r, lw, fa, fb, g);       \
  pull_level2<7, B, kMode>(a, sm, so, cm, xw, r, lw, fa, fb, g);       \
  pull_level2<8, B, kMode>(a, sm, so, cm, xw, r, lw, fa, fb, g);
        if (any_link<kMode>(lw)) {
          TLB_PULL2(true)
        } else {
          TLB_PULL2(false)
        }
#undef TLB_PULL2
        if constexpr ((kMode & kModeMoving) != 0) {
          // moving flat walls (Sec. 2.2): the bounced diagonal links of rows
          // 0 and ly - 1 gain 6 w_i rho_w c_ix u_w, rho_w the node's own
          // zeroth moment at the intermediate level
          if (r == 0 || r == ly - 1) {
            const Mom4<C>* m = sm[so][cm];
            const C rwa = m[0].rho, rwb = m[1].rho;
            if (r == 0) {
              const C k = C(6) * w_dir<C>(5) * a.uw0;
              fa[5] += k * rwa;
              fb[5] += k * rwb;
              fa[6] -= k * rwa;
              fb[6] -= k * rwb;
            }
            if (r == ly - 1) {
              const C k = C(6) * w_dir<C>(8) * a.uw1;
              fa[8] += k * rwa;
              fb[8] += k * rwb;
              fa[7] -= k * rwa;
              fb[7] -= k * rwb;
            }
          }
        }
        kw[0] = sum9(fa);
        kw[1] = sum9(fb);
        kw[2] = momentum_x(fa, fb);
        kw[3] = momentum_y(fa, fb);
        kw[4] = sum9(g);
        ra = kw[0];
        rb = kw[1];
        pa = psi_of<St>(ra, a.rho0, a.inv_rho0);
        pb = psi_of<St>(rb, a.rho0, a.inv_rho0);
      }
    }
    const int s = ring_slot<R1>(r);
    s2_rho[0][s][c1] = ra;
    s2_rho[1][s][c1] = rb;
    s2_psi[0][s][c1] = pa;
    s2_psi[1][s][c1] = pb;
  };

  // Level 2, phase 2: collision of row r and the 27 stores of f*(t+2).
  auto level2_collide = [&](int r, const C (&ku)[5], uint32_t lu) {
    const O yrow = (O)r * row_b;
    if (kSolid && (lu & kSelfSolid)) {
#pragma unroll
      for (int p = 0; p < 27; ++p) {
        if (St::kRest32 && p % 9 == 0) mdst.str(rest_off<St>(Lo, p / 9, r), Lo.v0r, 0.0f);
        else mdst.st((O)p * plane_b + yrow, Lo.v0, C(0));
      }
      return;
    }
    const C Da = ku[0], Db = ku[1], jx = ku[2], jy = ku[3], Dt = ku[4];
    const C ra = Da, rb = Db, temp = Dt;
    if constexpr (kTop) {
      if (top_chunk && r == ly - 1) top_sum[1] += (double)temp - (double)a.t_top;
    }
    if constexpr (kMoments) put_moments(1, r, Da, Db, jx, jy, Dt);
    int rs[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) rs[d] = ring_slot<R1>(r - 2 + d);
    C FA[2], FB[2];
    step2_forces(a, s2_rho, s2_psi, rs, c1, ra, rb, temp, FA, FB);
    const C rho = ra + rb;
    const C inv_rho = recip<St>(rho);
    const C ux = jx * inv_rho, uy = jy * inv_rho;
    const C Fx = FA[0] + FB[0], Fy = FA[1] + FB[1];
    const C hx = ux + C(0.5) * Fx * inv_rho;
    const C hy = uy + C(0.5) * Fy * inv_rho;
    const C tA = a.tau * recip<St>(ra), tB = a.tau * recip<St>(rb);
    const C uax = ux + FA[0] * tA, uay = uy + FA[1] * tA;
    const C ubx = ux + FB[0] * tB, uby = uy + FB[1] * tB;
    const C ua2 = uax * uax + uay * uay;
    const C ub2 = ubx * ubx + uby * uby;
    const C uh2 = hx * hx + hy * hy;
    C sa = 0, sb = 0, sg = 0;
    const O p9 = plane_b * 9, p18 = plane_b * 18;
#define TLB_PAIR2(I)                                        \
  {                                                         \
    constexpr int J = Dir<I>::opp;                          \
    C Sa, Dla, Sb, Dlb, Sg, Dlg;                            \
    eq_even_odd<I>(ra, uax, uay, ua2, Sa, Dla);             \
    eq_even_odd<I>(rb, ubx, uby, ub2, Sb, Dlb);             \
    eq_even_odd<I>(temp, hx, hy, uh2, Sg, Dlg);             \
    if constexpr (St::kDev) {                               \
      constexpr C w = w_dir<C>(I);                          \
      Sa -= w * a.ref_a;                                    \
      Sb -= w * a.ref_b;                                    \
      Sg -= w * a.ref_t;                                    \
    }                                                       \
    const C eaI = St::stored(Sa + Dla), eaJ = St::stored(Sa - Dla); \
    const C ebI = St::stored(Sb + Dlb), ebJ = St::stored(Sb - Dlb); \
    const C egI = St::stored(Sg + Dlg), egJ = St::stored(Sg - Dlg); \
    sa += eaI + eaJ;                                        \
    sb += ebI + ebJ;                                        \
    sg += egI + egJ;                                        \
    const O oI = (O)I * plane_b + yrow, oJ = (O)J * plane_b + yrow; \
    mdst.st(oI, Lo.v0, eaI);                                \
    mdst.st(oJ, Lo.v0, eaJ);                                \
    mdst.st(oI + p9, Lo.v0, ebI);                           \
    mdst.st(oJ + p9, Lo.v0, ebJ);                           \
    mdst.st(oI + p18, Lo.v0, egI);                          \
    mdst.st(oJ + p18, Lo.v0, egJ);                          \
  }
    TLB_PAIR2(1) TLB_PAIR2(2) TLB_PAIR2(5) TLB_PAIR2(6)
#undef TLB_PAIR2
    if constexpr (St::kRest32) {
      // FP32 remainders of the rounded moving deviations
      mdst.str(rest_off<St>(Lo, 0, r), Lo.v0r, (Da - a.ref_a) - sa);
      mdst.str(rest_off<St>(Lo, 1, r), Lo.v0r, (Db - a.ref_b) - sb);
      mdst.str(rest_off<St>(Lo, 2, r), Lo.v0r, (Dt - a.ref_t) - sg);
    } else {
      mdst.st(yrow, Lo.v0, Da - sa);
      mdst.st(yrow + p9, Lo.v0, Db - sb);
      mdst.st(yrow + p18, Lo.v0, Dt - sg);
    }
  };

  // One row iteration (see the header): ra = first + dir k.
  const int dir = down ? -1 : 1;
  const int first = down ? y1 - 1 + 5 : y0 - 5;
  uint32_t pm1 = mask_of(first), pm2 = mask_of(first - 4 * dir);
  auto in_rows = [&](int r, int lo, int hi) { return r >= lo && r < hi && r >= 0 && r < ly; };
  auto iterate = [&](int k, C (&k1w)[4], uint32_t& l1w, const C (&k1u)[4], uint32_t l1u,
                     C (&k2w)[5], uint32_t& l2w, const C (&k2u)[5], uint32_t l2u) {
    const int ra = first + dir * k;
    const int rb = ra - 2 * dir, rc = ra - 4 * dir, rd = ra - 6 * dir;
    const bool do_a = ra >= y0 - 5 && ra < y1 + 5;
    const bool do_b = in_rows(rb, y0 - 3, y1 + 3) && !(kSolid && (l1u & kSelfSolid));
    const bool do_c = rc >= y0 - 2 && rc < y1 + 2;
    const bool do_d = out_lane && rd >= y0 && rd < y1;
    // masks of rows ra and rc (loaded during the previous iteration), then
    // the loads of the next iteration's
    const uint32_t ma = pm1, mc = pm2;
    pm1 = mask_of(ra + dir);
    pm2 = mask_of(rc + dir);
    // phase 1: HBM loads first, then the LDS work of level 2
    C f[18], g[9];
    if (do_a) level1_pull(ra, ma, f, l1w);
    if (do_b) pull_thermal<St, kMode>(a, msrc, Lo, xw, rb, l1u, g);
    if (do_c) level2_density(rc, mc, k2w, l2w);
    if (do_a) level1_density(ra, f, l1w, k1w);
    __syncthreads();
    // phase 2
    if (do_b) level1_moments(rb, k1u, g);
    if (do_d) level2_collide(rd, k2u, l2u);
    __syncthreads();
  };

  C f0[4], f1[4], f2[4];
  C h0[5], h1[5], h2[5];
  uint32_t l0 = kSelfSolid, l1 = kSelfSolid, l2 = kSelfSolid;
  uint32_t m0 = kSelfSolid, m1 = kSelfSolid, m2 = kSelfSolid;
  const int n_iter = ((y1 - y0) + 11 + 2) / 3 * 3;
  for (int k = 0; k < n_iter; k += 3) {
    iterate(k, f0, l0, f1, l1, h0, m0, h1, m1);
    iterate(k + 1, f1, l1, f2, l2, h1, m1, h2, m2);
    iterate(k + 2, f2, l2, f0, l0, h2, m2, h0, m0);
  }

  if constexpr (kTop) {
    // fixed-order block sums into partials[level * strips + strip]
    if (top_chunk) {
      __shared__ double s_top[2][BT / 64];
#pragma unroll
      for (int lev = 0; lev < 2; ++lev) {
        double v = top_sum[lev];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if ((tid & 63) == 0) s_top[lev][tid >> 6] = v;
      }
      __syncthreads();
      if (tid < 2) {
        double v = 0;
        for (int w = 0; w < BT / 64; ++w) v += s_top[tid][w];
        a.partials[(size_t)tid * nbx + (tile - chunk * nbx)] = v;
      }
    }
  }
}

}  // namespace tlbk
