// Discrete adjoint of the lattice Boltzmann step (flat walls, FP64/FP32
// storage), for the gradient of the time-averaged top-wall Nusselt number
// with respect to the bottom-wall temperature profile T_b(x).
//
// Forward map of one step at a fluid node x (Sec. 2): pull the populations
// (bounce-back / anti-bounce-back at the walls, the bottom one at T_b),
// moments rho_l, j, T; forces F_l from the pseudopotentials of the 5 x 5
// neighbourhood (Eqs. (7), (10)-(12)) plus buoyancy (Eq. (22)); u = j/rho,
// u_l = u + tau F_l / rho_l (Eq. (6)), u^H = u + F / (2 rho); BGK towards
// f^eq(rho_l, u_l), g^eq(T, u^H) (Eqs. (2), (3), (16), (18)).
//
// Reverse sweep for one step, given lambda(t+1) = dL/d f*(t+1):
//   adj_local    per node: adjoint of the BGK relaxation, the equilibria, the
//                velocity shift, u^H, u = j/rho, the node's own terms of the
//                forces and the moments -> dL/d f(t) pulled values (local
//                part) and dL/dF_l;
//   adj_scatter  per node: the transpose of the force stencils (the node's
//                density enters its neighbours' forces) -> dL/drho_l;
//   adj_pull     per node: the transpose of the pull (each post-collision
//                value is pulled exactly once) -> lambda(t); its bottom-row
//                blocks also take the anti-bounce-back source 2 w_i T_b of
//                the bottom links -> dL/dT_b per column; where the next
//                reverse step's state is at hand it also does that step's
//                adj_density.
// Densities and pseudopotentials of the step's pulled state are precomputed
// by adj_density; the forward quantities of a node are recomputed from them
// and from the node's pulled populations.
//
// tau = tau_g = 1 (kTauOne): the relaxation passes nothing of lambda(t+1)
// straight through, so dL/d f_{l,i}(t) at a node is rbar_l + c_i.jbar and
// dL/d g_i(t) is tbar, five numbers per node: adj_local writes those (planes
// 0..4 of fbar: rbar_A, rbar_B, jbar_x, jbar_y, tbar) instead of 27 values,
// adj_scatter adds the stencil transpose to rbar_l, and the next reverse
// step's adj_local gathers lambda from the five numbers of each source node
// (no adj_pull; adj_scatter takes over its T_b gradient and densities).
#pragma once

#include "lb_kernels.hpp"

namespace tlbk {

template <typename C>
struct AdjArgs {
  StepArgs<C> s;         // forward arguments (walls, constants, layout)
  const void* state;     // f*(t) (stored type)
  const C* lam_next;     // lambda(t+1), population layout
  C* lam;                // lambda(t), population layout
  C* fbar;               // dL/d f(t) pulled values (27 planes)
  C* Fbar;               // dL/dF: 4 planes (F_A,x F_A,y F_B,x F_B,y)
  C* aux;                // rho_A, rho_B, psi_A, psi_B of the pulled state
  C* rbar;               // dL/drho from the stencil transpose (2 planes)
  double* grad;          // [lx] accumulated dL/dT_b
  double* loss_terms;    // per-step loss terms (forward)
  const void* next_state;  // state of the next reverse step, or null: adj_pull
                           // then also fills its aux (tau != 1)
  // tau = 1: moments rho_A, rho_B, j_x, j_y, T of this step's pulled state
  // and of the next reverse step's ([5] planes, population layout; mom_next
  // null: not at hand), from the taped run instead of the states
  const C* mom;
  const C* mom_next;
  C kappa_top;           // dL/dT of each top-row node for this step
  int step_index;
  int loss_stride;       // slots per step in loss_terms
  // tau = 1: the compact planes (fbar) and dL/drho (rbar) of the previous
  // reverse step (time t+1), from which adj_local gathers lambda(t+1), or
  // have_prev = 0 at the first reverse step (lambda = 0); aux_next receives
  // the densities of next_state
  const C* cmp_prev;
  const C* rbar_prev;
  C* aux_next;
  int have_prev;
};

// Element index of plane p at node (x, y) in a population-layout array. The
// adjoint runs only on population buffers below 4 GiB (27 planes), so every
// index of its arrays fits in 32 bits, which keeps the neighbour addressing
// of the stencil transposes cheap.
template <typename C>
__device__ inline uint32_t plane_index(const StepArgs<C>& a, int p, int x, int y) {
  return (uint32_t)p * (uint32_t)a.pop_stride + (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
}

template <typename C>
__device__ inline int wrapx(const StepArgs<C>& a, int x) {
  return x < 0 ? x + a.lx : (x >= a.lx ? x - a.lx : x);
}

// LDS tile of the stencil kernels: a block of 256 threads owns 64 x 4
// nodes and stages NF fields of the (64 + 4) x (4 + 4) cells within 2 of
// them (x periodic; rows beyond the walls take `wall`), so the 5 x 5
// stencils of adj_local and adj_scatter read LDS instead of global memory.
constexpr int kAdjTX = 64, kAdjTY = 4, kAdjHalo = 2;
constexpr int kAdjTW = kAdjTX + 2 * kAdjHalo, kAdjTH = kAdjTY + 2 * kAdjHalo;

template <typename C, int NF>
struct AdjTile {
  C v[NF][kAdjTH][kAdjTW];
};

// Lattice column of tile column x (x >= -kAdjHalo, lx >= 3): one period
// folds it, except on lattices narrower than a tile.
__device__ inline int tile_column(int x, int lx) {
  if (x < 0) x += lx;
  if (x >= lx) x = x - lx < lx ? x - lx : x % lx;
  return x;
}

// Fill the tile of the block at (x0, y0): field f of cell (cx, cy) is
// load(f, x, y) at the lattice node (x, y), or wall[f] outside the rows.
template <typename C, int NF, class Load>
__device__ inline void fill_tile(AdjTile<C, NF>& t, int x0, int y0, int lx, int ly,
                                 const C (&wall)[NF], Load load) {
  for (int c = threadIdx.x; c < kAdjTW * kAdjTH; c += 256) {
    const int cx = c % kAdjTW, cy = c / kAdjTW;
    const int x = tile_column(x0 - kAdjHalo + cx, lx), y = y0 - kAdjHalo + cy;
    const bool in = y >= 0 && y < ly;
#pragma unroll
    for (int f = 0; f < NF; ++f) t.v[f][cy][cx] = in ? load(f, x, y) : wall[f];
  }
}

// Pulled populations of node (x, y) from the state (flat walls).
template <class St>
__device__ inline void adj_pull_node(const AdjArgs<typename St::C>& a, int x, int y,
                                     typename St::C (&f)[18], typename St::C (&g)[9]) {
  using O = Off<0>;
  const O row_b = (O)a.s.pitch * sizeof(typename St::T);
  const O plane_b = (O)a.s.pop_stride * sizeof(typename St::T);
  const uint32_t lm = link_mask<0u>(a.s, x, y);
  const PopMem<St, 0u> m(a.state, (uint64_t)plane_b * 27);
  const LaneOff<0u> L = lane_off<St, 0u>(x, a.s.lx, plane_b, row_b);
  pull_fluid<St, 0u>(a.s, m, L, y, lm, f);
  pull_thermal<St, 0u>(a.s, m, L, x, y, lm, g);
}

// Pulled temperature populations of node (x, y) only (flat walls).
template <class St>
__device__ inline void adj_pull_thermal_node(const AdjArgs<typename St::C>& a, int x, int y,
                                             typename St::C (&g)[9]) {
  using O = Off<0>;
  const O row_b = (O)a.s.pitch * sizeof(typename St::T);
  const O plane_b = (O)a.s.pop_stride * sizeof(typename St::T);
  const uint32_t lm = link_mask<0u>(a.s, x, y);
  const PopMem<St, 0u> m(a.state, (uint64_t)plane_b * 27);
  const LaneOff<0u> L = lane_off<St, 0u>(x, a.s.lx, plane_b, row_b);
  pull_thermal<St, 0u>(a.s, m, L, x, y, lm, g);
}

// Densities and pseudopotentials of `state` pulled at node (x, y), into out
// (4 planes: rho_A, rho_B, psi_A, psi_B).
template <class St>
__device__ inline void density_node(const AdjArgs<typename St::C>& a, const void* state, int x,
                                    int y, typename St::C* out) {
  using C = typename St::C;
  using O = Off<0>;
  const O row_b = (O)a.s.pitch * sizeof(typename St::T);
  const O plane_b = (O)a.s.pop_stride * sizeof(typename St::T);
  const uint32_t lm = link_mask<0u>(a.s, x, y);
  const PopMem<St, 0u> m(state, (uint64_t)plane_b * 27);
  const LaneOff<0u> L = lane_off<St, 0u>(x, a.s.lx, plane_b, row_b);
  C f[18];
  pull_fluid<St, 0u>(a.s, m, L, y, lm, f);
  const C ra = sum9(f), rb = sum9(f + 9);
  out[plane_index(a.s, 0, x, y)] = ra;
  out[plane_index(a.s, 1, x, y)] = rb;
  out[plane_index(a.s, 2, x, y)] = psi_exp(ra, a.s.rho0, a.s.inv_rho0);
  out[plane_index(a.s, 3, x, y)] = psi_exp(rb, a.s.rho0, a.s.inv_rho0);
}

template <class St>
__global__ __launch_bounds__(256) void adj_density(AdjArgs<typename St::C> a) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  if (x >= a.s.lx) return;
  density_node<St>(a, a.state, x, y, a.aux);
}

// The same from a moment-tape slot (tau = 1).
template <typename C>
__device__ inline void density_from_moments(const AdjArgs<C>& a, const C* mom, int x, int y,
                                            C* out) {
  const C ra = mom[plane_index(a.s, 0, x, y)], rb = mom[plane_index(a.s, 1, x, y)];
  out[plane_index(a.s, 0, x, y)] = ra;
  out[plane_index(a.s, 1, x, y)] = rb;
  out[plane_index(a.s, 2, x, y)] = psi_exp(ra, a.s.rho0, a.s.inv_rho0);
  out[plane_index(a.s, 3, x, y)] = psi_exp(rb, a.s.rho0, a.s.inv_rho0);
}

template <class St>
__global__ __launch_bounds__(256) void adj_density_moments(AdjArgs<typename St::C> a) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  if (x >= a.s.lx) return;
  density_from_moments(a, a.mom, x, y, a.aux);
}

// Forward loss term of one step: sum over the top row of T - T_top from the
// pulled state, in a fixed order (one block).
template <class St>
__global__ __launch_bounds__(256) void adj_top_row_sum(AdjArgs<typename St::C> a) {
  using C = typename St::C;
  __shared__ double part[256];
  double acc = 0;
  const int y = a.s.ly - 1;
  for (int x = threadIdx.x; x < a.s.lx; x += 256) {
    C g[9];
    adj_pull_thermal_node<St>(a, x, y, g);
    acc += (double)sum9(g) - (double)a.s.t_top;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  // slot 0 of the step's row; the other slots (per-strip sums of the fused
  // kernel's steps) are zero here
  double* row = a.loss_terms + (size_t)a.step_index * a.loss_stride;
  if (threadIdx.x == 0) row[0] = part[0];
  for (int k = 1 + threadIdx.x; k < a.loss_stride; k += 256) row[k] = 0.0;
}

// Compact planes of the tau = 1 form (in the fbar array).
constexpr int kCompactRbar = 0, kCompactJx = 2, kCompactJy = 3, kCompactT = 4;

// Weighted moments of nine values v_i over the D2Q9 directions: sum w_i v_i,
// sum w_i v_i c_i and the three distinct entries of sum w_i v_i c_i c_i.
template <typename C>
struct WMom {
  C m0, mx, my, mxx, myy, mxy;
};

template <typename C>
__device__ inline WMom<C> weighted_moments(const C* v) {
  constexpr C w0 = w_c2<C>(0), w1 = w_c2<C>(1), w2 = w_c2<C>(2);
  const C ax = v[1] + v[3], ay = v[2] + v[4];
  const C dp = v[5] + v[7], dm = v[6] + v[8];
  const C d = dp + dm;
  const C r = v[5] - v[7];
  WMom<C> m;
  m.m0 = w0 * v[0] + w1 * (ax + ay) + w2 * d;
  m.mx = w1 * (v[1] - v[3]) + w2 * (r + (v[8] - v[6]));
  m.my = w1 * (v[2] - v[4]) + w2 * (r + (v[6] - v[8]));
  m.mxx = w1 * ax + w2 * d;
  m.myy = w1 * ay + w2 * d;
  m.mxy = w2 * (dp - dm);
  return m;
}

// Adjoint of the equilibrium w_i rho (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u^2)
// (Eqs. (2), (3), (16)): given the weighted moments m of the sensitivities
// of the nine values, adds d/drho to rbar and d/du to ubar.
template <typename C>
__device__ inline void eq_adjoint(const WMom<C>& m, C rho, C ux, C uy, C& rbar, C& ubx, C& uby) {
  const C qx = m.mxx * ux + m.mxy * uy, qy = m.mxy * ux + m.myy * uy;
  const C u2 = ux * ux + uy * uy;
  rbar += m.m0 * (C(1) - C(1.5) * u2) + C(3) * (m.mx * ux + m.my * uy) + C(4.5) * (qx * ux + qy * uy);
  ubx += rho * (C(3) * m.mx + C(9) * qx - C(3) * ux * m.m0);
  uby += rho * (C(3) * m.my + C(9) * qy - C(3) * uy * m.m0);
}

// Pair-difference sums of a 5 x 5 stencil of tile field v around (cy0, cx0):
// sum over c != 0 of p(|c|^2) v(x + c) c (q) and of the nearest-neighbour
// w(|c|^2) v(x + c) c (n), each pair c, -c as one difference.
template <typename C, int NF>
__device__ inline void stencil_sums(const AdjTile<C, NF>& t, int f, int cy0, int cx0, C (&q)[2],
                                    C (&n)[2]) {
  q[0] = q[1] = n[0] = n[1] = C(0);
#pragma unroll
  for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
    for (int dx = 1; dx <= 2; ++dx) {
      const int c2 = dx * dx + dy * dy;
      const C diff = t.v[f][cy0 + dy][cx0 + dx] - t.v[f][cy0 + dy][cx0 - dx];
      q[0] += (p_c2<C>(c2) * C(dx)) * diff;
      if (c2 <= 2) n[0] += (w_c2<C>(c2) * C(dx)) * diff;
    }
#pragma unroll
  for (int dx = -2; dx <= 2; ++dx)
#pragma unroll
    for (int dy = 1; dy <= 2; ++dy) {
      const int c2 = dx * dx + dy * dy;
      const C diff = t.v[f][cy0 + dy][cx0 + dx] - t.v[f][cy0 - dy][cx0 + dx];
      q[1] += (p_c2<C>(c2) * C(dy)) * diff;
      if (c2 <= 2) n[1] += (w_c2<C>(c2) * C(dy)) * diff;
    }
}

// Nearest-neighbour sum of w(|c|^2) v(x + c) c only.
template <typename C, int NF>
__device__ inline void nn_sums(const AdjTile<C, NF>& t, int f, int cy0, int cx0, C (&n)[2]) {
  n[0] = n[1] = C(0);
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
    n[0] += w_c2<C>(1 + dy * dy) * (t.v[f][cy0 + dy][cx0 + 1] - t.v[f][cy0 + dy][cx0 - 1]);
#pragma unroll
  for (int dx = -1; dx <= 1; ++dx)
    n[1] += w_c2<C>(1 + dx * dx) * (t.v[f][cy0 + 1][cx0 + dx] - t.v[f][cy0 - 1][cx0 + dx]);
}

// Tile fields of adj_local: densities and pseudopotentials of the pulled
// state (0..3), and at tau = 1 the previous reverse step's dL/drho_l (4, 5),
// jbar (6, 7) and tbar (8) from which lambda(t+1) is gathered.
constexpr int kLocRho = 0, kLocPsi = 2, kLocR = 4, kLocJ = 6, kLocT = 8;

template <class St, bool kTauOne>
__global__ __launch_bounds__(256) void adj_local(AdjArgs<typename St::C> a) {
  using C = typename St::C;
  const StepArgs<C>& s = a.s;
  constexpr int NF = kTauOne ? 9 : 4;
  __shared__ AdjTile<C, NF> tile;
  const int x0 = blockIdx.x * kAdjTX, y0 = blockIdx.y * kAdjTY;
  const int tx = threadIdx.x % kAdjTX, ty = threadIdx.x / kAdjTX;
  const int x = x0 + tx, y = y0 + ty;
  const bool valid = x < s.lx && y < s.ly;
  // tau = 1: the node's taped moments, loaded before the tile so that the
  // two latencies overlap
  C mo[5] = {0, 0, 0, 0, 0};
  if constexpr (kTauOne) {
    if (valid) {
#pragma unroll
      for (int k = 0; k < 5; ++k) mo[k] = a.mom[plane_index(s, k, x, y)];
    }
  }
  {
    // wall rows: the wetting densities; no lambda is gathered from them
    C wall[NF] = {s.rho_wall0, s.rho_wall1, psi_exp(s.rho_wall0, s.rho0, s.inv_rho0),
                  psi_exp(s.rho_wall1, s.rho0, s.inv_rho0)};
    for (int f = 4; f < NF; ++f) wall[f] = C(0);
    const bool prev = a.have_prev != 0;
    fill_tile(tile, x0, y0, s.lx, s.ly, wall, [&](int f, int xx, int yy) -> C {
      if (f < 4) return a.aux[plane_index(s, f, xx, yy)];
      if (!prev) return C(0);
      return f < kLocJ ? a.rbar_prev[plane_index(s, f - kLocR, xx, yy)]
                       : a.cmp_prev[plane_index(s, kCompactJx + f - kLocJ, xx, yy)];
    });
  }
  __syncthreads();
  if (!valid) return;
  const int cx0 = tx + kAdjHalo, cy0 = ty + kAdjHalo;

  // ---- forward recompute: the moments of the pulled state (taped at tau =
  // 1, else pulled from the state)
  C ra, rb, temp, jx, jy;
  if constexpr (kTauOne) {
    ra = mo[0];
    rb = mo[1];
    jx = mo[2];
    jy = mo[3];
    temp = mo[4];
  } else {
    C f[18], g[9];
    adj_pull_node<St>(a, x, y, f, g);
    ra = sum9(f);
    rb = sum9(f + 9);
    temp = sum9(g);
    jx = momentum_x(f, f + 9);
    jy = momentum_y(f, f + 9);
  }
  const C rl[2] = {ra, rb};
  const C inv_rl[2] = {C(1) / ra, C(1) / rb};
  const C inv_rho = C(1) / (ra + rb);
  const C ux = jx * inv_rho, uy = jy * inv_rho;
  // Sr: 25-point sums of psi_l, Sa: nearest-neighbour sums of psi_l, X:
  // nearest-neighbour sums of the other component's density
  C Sa[2][2], Sr[2][2], X[2][2], ps[2], dps[2];
  for (int l = 0; l < 2; ++l) {
    ps[l] = tile.v[kLocPsi + l][cy0][cx0];
    dps[l] = C(1) - ps[l] * s.inv_rho0;  // d psi / d rho = exp(-rho / rho0)
    stencil_sums(tile, kLocPsi + l, cy0, cx0, Sr[l], Sa[l]);
    nn_sums(tile, kLocRho + 1 - l, cy0, cx0, X[l]);
  }
  const C gcross = s.g12 * s.inv_rho0 * s.inv_rho0;
  const C ga[2] = {s.ga0, s.ga1}, gr[2] = {s.gr0, s.gr1};
  C F[2][2];
  for (int l = 0; l < 2; ++l)
    for (int d = 0; d < 2; ++d)
      F[l][d] = -ps[l] * (ga[l] * Sa[l][d] + gr[l] * Sr[l][d]) - gcross * rl[l] * X[l][d];
  F[0][1] += ra * s.alpha_g * temp;
  F[1][1] += rb * s.alpha_g * temp;
  const C Fx = F[0][0] + F[1][0], Fy = F[0][1] + F[1][1];
  C ul[2][2];
  for (int l = 0; l < 2; ++l) {
    ul[l][0] = ux + s.tau * F[l][0] * inv_rl[l];
    ul[l][1] = uy + s.tau * F[l][1] * inv_rl[l];
  }
  const C hx = ux + Fx * C(0.5) * inv_rho, hy = uy + Fy * C(0.5) * inv_rho;

  // ---- lambda(t+1) of the node: loaded, or at tau = 1 gathered from the
  // previous reverse step's compact values (the transpose of the pull: the
  // population this node streamed in direction i was pulled by x + c_i, or
  // bounced back into the node itself across a wall)
  C lamv[27];
  if constexpr (kTauOne) {
    const bool lo = y == 0, hi = y == s.ly - 1;
    const C rA = tile.v[kLocR][cy0][cx0], rB = tile.v[kLocR + 1][cy0][cx0];
    const C Jx = tile.v[kLocJ][cy0][cx0], Jy = tile.v[kLocJ + 1][cy0][cx0];
    const C tt = tile.v[kLocT][cy0][cx0];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int cx = dir_cx(i), cy = dir_cy(i);
      const int ny = cy0 + cy, nx = cx0 + cx;
      const C cj = C(cx) * tile.v[kLocJ][ny][nx] + C(cy) * tile.v[kLocJ + 1][ny][nx];
      C la = tile.v[kLocR][ny][nx] + cj, lb = tile.v[kLocR + 1][ny][nx] + cj;
      C lt = tile.v[kLocT][ny][nx];
      if (cy != 0) {
        // across a wall: the node's own values in direction opp(i)
        const bool wall = cy < 0 ? lo : hi;
        const C oj = C(cx) * Jx + C(cy) * Jy;
        la = wall ? rA - oj : la;
        lb = wall ? rB - oj : lb;
        lt = wall ? -tt : lt;
      }
      lamv[i] = la;
      lamv[9 + i] = lb;
      lamv[18 + i] = lt;
    }
  } else {
#pragma unroll
    for (int p = 0; p < 27; ++p) lamv[p] = a.lam_next[plane_index(s, p, x, y)];
  }

  // ---- adjoint of the BGK relaxation and of the equilibria: the
  // equilibria take (1 - ka) lambda, the kept part ka lambda (zero at tau = 1)
  C rbar[2] = {0, 0}, ubar[2][2] = {{0, 0}, {0, 0}}, tbar = 0, hbar[2] = {0, 0};
  {
    WMom<C> m[3] = {weighted_moments(lamv), weighted_moments(lamv + 9), weighted_moments(lamv + 18)};
    if constexpr (!kTauOne) {
      for (int k = 0; k < 3; ++k) {
        const C e = k < 2 ? s.inv_tau : s.inv_tau_g;
        m[k] = {e * m[k].m0, e * m[k].mx, e * m[k].my, e * m[k].mxx, e * m[k].myy, e * m[k].mxy};
      }
    }
    eq_adjoint(m[0], ra, ul[0][0], ul[0][1], rbar[0], ubar[0][0], ubar[0][1]);
    eq_adjoint(m[1], rb, ul[1][0], ul[1][1], rbar[1], ubar[1][0], ubar[1][1]);
    eq_adjoint(m[2], temp, hx, hy, tbar, hbar[0], hbar[1]);
  }
  // ---- velocities: u_l = u + tau F_l / rho_l, u^H = u + F / (2 rho), u = j / rho
  C Fbar[2][2];
  const C uc[2] = {ubar[0][0] + ubar[1][0] + hbar[0], ubar[0][1] + ubar[1][1] + hbar[1]};
  const C hh = C(0.5) * inv_rho;
  for (int l = 0; l < 2; ++l) {
    const C ti = s.tau * inv_rl[l];
    for (int d = 0; d < 2; ++d) Fbar[l][d] = ti * ubar[l][d] + hbar[d] * hh;
    rbar[l] -= ti * inv_rl[l] * (ubar[l][0] * F[l][0] + ubar[l][1] * F[l][1]);
  }
  const C rtot = -(hbar[0] * Fx + hbar[1] * Fy) * hh * inv_rho -
                 (uc[0] * jx + uc[1] * jy) * inv_rho * inv_rho;
  const C jbx = uc[0] * inv_rho, jby = uc[1] * inv_rho;
  rbar[0] += rtot;
  rbar[1] += rtot;
  // ---- the node's own terms of the forces
  for (int l = 0; l < 2; ++l) {
    // buoyancy rho_l alpha_g T e_y
    rbar[l] += Fbar[l][1] * s.alpha_g * temp;
    tbar += Fbar[l][1] * s.alpha_g * rl[l];
    // cross-force prefactor rho_l / rho0
    rbar[l] -= gcross * (Fbar[l][0] * X[l][0] + Fbar[l][1] * X[l][1]);
    // self-force prefactor psi_l(x)
    const C psibar = -(Fbar[l][0] * (ga[l] * Sa[l][0] + gr[l] * Sr[l][0]) +
                       Fbar[l][1] * (ga[l] * Sa[l][1] + gr[l] * Sr[l][1]));
    rbar[l] += psibar * dps[l];
  }
  // ---- moments (and the loss term of the top row: dL/dT = kappa_top)
  if (y == s.ly - 1) tbar += a.kappa_top;
  for (int l = 0; l < 2; ++l)
    for (int d = 0; d < 2; ++d) a.Fbar[plane_index(s, 2 * l + d, x, y)] = Fbar[l][d];
  if constexpr (kTauOne) {
    a.fbar[plane_index(s, kCompactRbar, x, y)] = rbar[0];
    a.fbar[plane_index(s, kCompactRbar + 1, x, y)] = rbar[1];
    a.fbar[plane_index(s, kCompactJx, x, y)] = jbx;
    a.fbar[plane_index(s, kCompactJy, x, y)] = jby;
    a.fbar[plane_index(s, kCompactT, x, y)] = tbar;
  } else {
    const C ka = C(1) - s.inv_tau, kg = C(1) - s.inv_tau_g;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const C cx = C(dir_cx(i)), cy = C(dir_cy(i));
      const C cj = cx * jbx + cy * jby;
      a.fbar[plane_index(s, i, x, y)] = ka * lamv[i] + (rbar[0] + cj);
      a.fbar[plane_index(s, 9 + i, x, y)] = ka * lamv[9 + i] + (rbar[1] + cj);
      a.fbar[plane_index(s, 18 + i, x, y)] = kg * lamv[18 + i] + tbar;
    }
  }
}

// dL/dT_b(c) += sum of 2 w_i gbar_i(x, 0) over the bottom links whose solid
// source lies in column c: i = 2 at x = c, i = 5 at x = c + 1, i = 6 at
// x = c - 1 (gbar = dL/d of the pulled g, complete once adj_local is done).
template <class St, bool kTauOne>
__device__ inline void grad_tb_column(const AdjArgs<typename St::C>& a, int c) {
  using C = typename St::C;
  const StepArgs<C>& s = a.s;
  // plane of gbar_i: its own, or the compact tbar (the same for every i)
  auto gp = [](int i) { return kTauOne ? kCompactT : 18 + i; };
  const double v = 2.0 * ((double)w_dir<C>(2) * (double)a.fbar[plane_index(s, gp(2), c, 0)] +
                          (double)w_dir<C>(5) * (double)a.fbar[plane_index(s, gp(5), wrapx(s, c + 1), 0)] +
                          (double)w_dir<C>(6) * (double)a.fbar[plane_index(s, gp(6), wrapx(s, c - 1), 0)]);
  a.grad[c] += v;
}

// Transpose of the force stencils: rho_l(x') enters the self forces of its
// 24 neighbours through psi_l and the cross forces of the other component's
// 8 neighbours through rho_l / rho0. With H_l = psi_l Fbar_l and K_l = rho_l
// Fbar_l of each node (formed as the tile is filled), dL/dpsi_l(x) gets
// -sum_c (ga_l w + gr_l p)(|c|^2) c.H_l(x - c) and dL/drho_{1-l}(x) gets
// -g12/rho0^2 sum_c w(|c|^2) c.K_l(x - c), each pair c, -c as one difference.
template <class St, bool kTauOne>
__global__ __launch_bounds__(256) void adj_scatter(AdjArgs<typename St::C> a) {
  using C = typename St::C;
  const StepArgs<C>& s = a.s;
  // H_A (x, y), H_B (x, y), K_A (x, y), K_B (x, y) of the tile and its
  // halo; zero beyond the walls (no force there)
  __shared__ AdjTile<C, 8> tile;
  const int x0 = blockIdx.x * kAdjTX, y0 = blockIdx.y * kAdjTY;
  const int tx = threadIdx.x % kAdjTX, ty = threadIdx.x / kAdjTX;
  const int x = x0 + tx, y = y0 + ty;
  const bool valid = x < s.lx && y < s.ly;
  // the node's own inputs, loaded before the tile so that the latencies
  // overlap: psi_l (for d psi / d rho), at tau = 1 its own dL/drho_l and the
  // next reverse step's densities
  C own_psi[2] = {0, 0}, own_rbar[2] = {0, 0}, next_rho[2] = {0, 0};
  if (valid) {
    own_psi[0] = a.aux[plane_index(s, 2, x, y)];
    own_psi[1] = a.aux[plane_index(s, 3, x, y)];
    if constexpr (kTauOne) {
      own_rbar[0] = a.fbar[plane_index(s, kCompactRbar, x, y)];
      own_rbar[1] = a.fbar[plane_index(s, kCompactRbar + 1, x, y)];
      if (a.mom_next) {
        next_rho[0] = a.mom_next[plane_index(s, 0, x, y)];
        next_rho[1] = a.mom_next[plane_index(s, 1, x, y)];
      }
    }
  }
  for (int c = threadIdx.x; c < kAdjTW * kAdjTH; c += 256) {
    const int cx = c % kAdjTW, cy = c / kAdjTW;
    const int xx = tile_column(x0 - kAdjHalo + cx, s.lx), yy = y0 - kAdjHalo + cy;
    const bool in = yy >= 0 && yy < s.ly;
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      C fx = 0, fy = 0, r = 0, p = 0;
      if (in) {
        fx = a.Fbar[plane_index(s, 2 * l, xx, yy)];
        fy = a.Fbar[plane_index(s, 2 * l + 1, xx, yy)];
        r = a.aux[plane_index(s, l, xx, yy)];
        p = a.aux[plane_index(s, 2 + l, xx, yy)];
      }
      tile.v[2 * l][cy][cx] = p * fx;
      tile.v[2 * l + 1][cy][cx] = p * fy;
      tile.v[4 + 2 * l][cy][cx] = r * fx;
      tile.v[5 + 2 * l][cy][cx] = r * fy;
    }
  }
  __syncthreads();
  if (!valid) return;
  const int cx0 = tx + kAdjHalo, cy0 = ty + kAdjHalo;
  const C gcross = s.g12 * s.inv_rho0 * s.inv_rho0;
  const C ga[2] = {s.ga0, s.ga1}, gr[2] = {s.gr0, s.gr1};
  C v[2];
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    // sum over pairs of coef(|c|^2) c.(H(x - c) - H(x + c)), half-plane c
    C acc = 0;
    auto pair = [&](int dx, int dy) {
      const int c2 = dx * dx + dy * dy;
      const C coef = ga[l] * w_c2<C>(c2) + gr[l] * p_c2<C>(c2);
      C dot = 0;
      if (dx != 0)
        dot = C(dx) * (tile.v[2 * l][cy0 - dy][cx0 - dx] - tile.v[2 * l][cy0 + dy][cx0 + dx]);
      if (dy != 0)
        dot += C(dy) * (tile.v[2 * l + 1][cy0 - dy][cx0 - dx] - tile.v[2 * l + 1][cy0 + dy][cx0 + dx]);
      acc += coef * dot;
    };
    pair(1, 0);
    pair(2, 0);
#pragma unroll
    for (int dy = 1; dy <= 2; ++dy)
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) pair(dx, dy);
    v[l] = -acc;
  }
  C cr[2];  // cross terms, by the component they act on
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    C acc = 0;
    auto pair = [&](int dx, int dy) {
      C dot = 0;
      if (dx != 0)
        dot = C(dx) * (tile.v[4 + 2 * l][cy0 - dy][cx0 - dx] - tile.v[4 + 2 * l][cy0 + dy][cx0 + dx]);
      if (dy != 0)
        dot += C(dy) * (tile.v[5 + 2 * l][cy0 - dy][cx0 - dx] - tile.v[5 + 2 * l][cy0 + dy][cx0 + dx]);
      acc += w_c2<C>(dx * dx + dy * dy) * dot;
    };
    pair(1, 0);
    pair(-1, 1);
    pair(0, 1);
    pair(1, 1);
    cr[1 - l] = -gcross * acc;
  }
  for (int l = 0; l < 2; ++l) {
    const C dps = C(1) - own_psi[l] * s.inv_rho0;
    C r = cr[l] + v[l] * dps;
    // tau = 1: the node's own dL/drho_l joins it (one plane to gather later)
    if constexpr (kTauOne) r = own_rbar[l] + r;
    a.rbar[plane_index(s, l, x, y)] = r;
  }
  if constexpr (kTauOne) {
    // no adj_pull at tau = 1 (the next adj_local gathers lambda): the bottom
    // row adds dL/dT_b of its columns here, and the next reverse step's
    // densities go to the other aux buffer
    if (y == 0) grad_tb_column<St, true>(a, x);
    if (a.mom_next) {
      a.aux_next[plane_index(s, 0, x, y)] = next_rho[0];
      a.aux_next[plane_index(s, 1, x, y)] = next_rho[1];
      a.aux_next[plane_index(s, 2, x, y)] = psi_exp(next_rho[0], s.rho0, s.inv_rho0);
      a.aux_next[plane_index(s, 3, x, y)] = psi_exp(next_rho[1], s.rho0, s.inv_rho0);
    }
  }
}

// Transpose of the pull: f*_i(y) was pulled by the node y + c_i, or, when
// that node is a wall, by y itself as direction opp(i) (bounce-back; with a
// minus sign for g, anti-bounce-back).
template <class St, bool kTauOne>
__global__ __launch_bounds__(256) void adj_pull(AdjArgs<typename St::C> a) {
  using C = typename St::C;
  const StepArgs<C>& s = a.s;
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  if (x >= s.lx) return;
  const int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  for (int i = 0; i < 9; ++i) {
    const int tx = wrapx(s, x + dir_cx(i)), ty = y + dir_cy(i);
    const bool wall = ty < 0 || ty >= s.ly;
    const int sx = wall ? x : tx, sy = wall ? y : ty, si = wall ? opp[i] : i;
    if constexpr (kTauOne) {
      // dL/d f_{l,si} = rbar_l + c_si.jbar, dL/d g_si = tbar at the source node
      const C jx = a.fbar[plane_index(s, kCompactJx, sx, sy)];
      const C jy = a.fbar[plane_index(s, kCompactJy, sx, sy)];
      const C cj = C(dir_cx(si)) * jx + C(dir_cy(si)) * jy;
      for (int l = 0; l < 2; ++l)
        a.lam[plane_index(s, 9 * l + i, x, y)] = a.rbar[plane_index(s, l, sx, sy)] + cj;
      const C gv = a.fbar[plane_index(s, kCompactT, sx, sy)];
      a.lam[plane_index(s, 18 + i, x, y)] = wall ? -gv : gv;
    } else {
      for (int l = 0; l < 2; ++l) {
        const C v = a.fbar[plane_index(s, 9 * l + si, sx, sy)] + a.rbar[plane_index(s, l, sx, sy)];
        a.lam[plane_index(s, 9 * l + i, x, y)] = v;
      }
      const C gv = a.fbar[plane_index(s, 18 + si, sx, sy)];
      a.lam[plane_index(s, 18 + i, x, y)] = wall ? -gv : gv;
    }
  }
  // the bottom row's blocks also accumulate dL/dT_b of their columns
  if (y == 0) grad_tb_column<St, kTauOne>(a, x);
  // densities of the next reverse step's state: aux is free again once
  // adj_local and adj_scatter of this step are done
  if (a.next_state) density_node<St>(a, a.next_state, x, y, a.aux);
}



}  // namespace tlbk
