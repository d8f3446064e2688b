/*
 * FP64 CPU oracle for the thermal two-component Shan-Chen lattice Boltzmann
 * update of TLBfind (arXiv:2109.12565).
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the CPU-baseline
 * timing leg of the benchmark link this file; the GPU library never does, and
 * the two share no code, header, table or helper.
 *
 * It is a plain, slow, step-by-step implementation of the scheme of Sec. 2,
 * written for a reader to check against the paper:
 *
 *   1. moments     rho_l = sum_i f_{l,i}; u = sum_{l,i} c_i f_{l,i} / rho;
 *                  T = sum_i g_i                  (Sec. 2.1 Eqs. (4)-(5);
 *                                                  Sec. 2.3 Eq. (17))
 *   2. pseudo-     psi_x = rho/rho0 for the cross force (Sec. 2.1 Eq. (8)),
 *      potentials  psi_s = rho0 (1 - exp(-rho/rho0)) for the self forces
 *                  (Sec. 2.1 Eq. (12)); solid nodes carry the wall
 *                  densities (Sec. 2.2.1).
 *   3. forces      F^x (Eq. (7)), F^a (Eq. (10)), F^r (Eq. (11)),
 *                  buoyancy rho_l alpha g T e_y (Sec. 2.3 Eq. (22));
 *                  F = sum_l F_l.
 *   4. velocities  u_l = u + tau F_l / rho_l (Eq. (6));
 *                  rho u^H = rho u + F/2 (Sec. 2.1, below Eq. (13)).
 *   5. collide     BGK (Eqs. (2), (16)) towards the second-order equilibria
 *                  f^eq(rho_l, u_l) (Eq. (3)) and g^eq(T, u^H) (Eq. (18)).
 *   6. stream      f(x + c_i, t+1) = f*(x, t) (Eqs. (1), (16)); a link whose
 *                  target is solid is reflected by half-way bounce-back
 *                  (Sec. 2.2) for f, and by anti-bounce-back holding the
 *                  wall temperature for g.
 *
 * Node loops run in parallel with OpenMP: every node's update depends only
 * on the previous state, so the thread count never changes a result; the
 * observable sums are serial, in row-major order.
 *
 * The state kept between steps is the pre-collision populations f(t), g(t);
 * streaming is done in push form (collide, then move), which is the same
 * arithmetic as the GPU's pull form reached by a different route.
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * project's design notes):
 *   - the repulsive coupling G^r enters with the sign the text gives (> 0);
 *   - the second component has its own couplings g_a[1], g_r[1];
 *   - two solid ghost rows per wall (the 25-point stencil reaches 2 rows);
 *   - walls are half-way: the wall plane lies half a cell beyond the last
 *     fluid row; solid cells are never collided nor streamed;
 *   - temperature walls: anti-bounce-back g_i(x,t+1) = -g*_{opp i}(x,t)
 *     + 2 w_i T_w, with T_w = t_bottom[column of the solid cell] for the
 *     bottom ghost rows and for solid cells flagged 1, and T_w = t_top for
 *     the top ghost rows and for solid cells flagged 2;
 *   - moving flat walls (Sec. 2.2, the Couette set-up of Sec. 3.2.2): the
 *     bottom and top walls move along x with u_wall[0], u_wall[1]; a link
 *     into a moving wall is bounced back with the momentum term of a wall
 *     moving at u_w, f_{opp i}(x,t+1) = f*_i(x,t) - 2 w_i rho_w (c_i.u_w)
 *     / cs^2, with rho_w the node's own density sum_j f*_{l,j}(x,t) (the
 *     terms cancel over the links of a flat wall, so mass is conserved),
 *     and g is anti-bounced against the even part of the equilibrium at
 *     the wall velocity, 2 w_i T_w (1 + (c_i.u_w)^2 / (2 cs^4) - u_w^2 /
 *     (2 cs^2)); solid cells inside the lattice do not move;
 *   - stress (Sec. 2.1 below Eq. (14), Sec. 3.2.2): the xy stress of a
 *     node is the viscous part -(1 - 1/(2 tau)) sum_l sum_i c_ix c_iy
 *     (f_{l,i} - f^eq_i(rho_l, u_l)) (the non-equilibrium the collision
 *     relaxes) minus the xy component of the interaction pressure tensor
 *     of the pseudopotential forces, 1/2 sum_l psi_l(x) sum_c G(c)
 *     psi(x + c) c_x c_y over the stencils and couplings of Eqs. (7),
 *     (10), (11);
 *   - Nu (Sec. 3.3.2 Eq. (24)) uses u^H, averages over fluid nodes, takes
 *     dT/dy by central differences with the mirror value 2 T_w - T at a
 *     solid neighbour, and normalises by kappa * dt_nominal / ly;
 *   - kinetic energy (Sec. 3.1) is the fluid-node mean of |u^H|^2.
 *
 * Parity: pinned by the tests under tests/ (closed forms, invariants and the
 * paper's printed phase-separation table of Appendix B).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9 velocities c_i and weights w_i (Sec. 2.1, Fig. 1(b)).
 * Order: rest, +x, +y, -x, -y, (+1,+1), (-1,+1), (-1,-1), (+1,-1). */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double WGT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                              1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

/* Weight w(c) of the nearest-neighbour shell, as a function of |c|^2
 * (Fig. 1(b): 4/9, 1/9, 1/36; zero beyond). */
static double w_of(int c2) {
  switch (c2) {
    case 0: return 4.0 / 9.0;
    case 1: return 1.0 / 9.0;
    case 2: return 1.0 / 36.0;
    default: return 0.0;
  }
}

/* Weight p(c) of the nearest + next-to-nearest shells, as a function of
 * |c|^2 (Fig. 1(b): the column headed |c_i| lists |c_i|^2). */
static double p_of(int c2) {
  switch (c2) {
    case 0: return 247.0 / 420.0;
    case 1: return 4.0 / 63.0;
    case 2: return 4.0 / 135.0;
    case 4: return 1.0 / 180.0;
    case 5: return 2.0 / 945.0;
    case 8: return 1.0 / 15120.0;
    default: return 0.0;
  }
}

typedef struct ora_params {
  int32_t lx, ly;
  int32_t periodic_y;   /* 1: y wraps (no walls); 0: solid walls below/above */
  int32_t pad_;
  double tau, tau_g;
  double rho0;
  double g12;
  double g_a[2];        /* short-range attraction G^a_{ll} (< 0) */
  double g_r[2];        /* mid-range repulsion G^r_{ll} (> 0) */
  double alpha_g;
  double t_top;
  double rho_wall[2];   /* wetting densities at solid nodes (Sec. 2.2.1) */
  double dt_nominal;    /* Delta T in the Nusselt normalisation */
  double u_wall[2];     /* x-velocity of the bottom and top walls */
} ora_params;

typedef struct ora_state {
  ora_params p;
  int64_t t;
  int nthreads;          /* threads of the parallel node loops */
  int n;                 /* lx * ly */
  double *f[2];          /* [9][n] pre-collision, per component */
  double *g;             /* [9][n] */
  uint8_t *solid;        /* [n] 0 fluid, 1 solid at t_bottom, 2 solid at t_top */
  double *t_bottom;      /* [lx] */
  /* work arrays */
  double *rho[2], *jx, *jy, *temp;
  double *fx[2], *fy[2]; /* force on each component */
  double *psi_s[2], *psi_x[2]; /* on a (ly+4) x lx grid with 2 ghost rows each side */
  double *fs[2], *gs;    /* post-collision */
  double *fn[2], *gn;    /* next pre-collision */
} ora_state;

static int wrapx(const ora_state *s, int x) {
  int lx = s->p.lx;
  while (x < 0) x += lx;
  while (x >= lx) x -= lx;
  return x;
}

/* Solid flag of lattice cell (x, y), y possibly outside [0, ly):
 * 0 fluid, 1 solid held at the bottom temperature, 2 at the top one. */
static int solid_at(const ora_state *s, int x, int y) {
  int ly = s->p.ly;
  x = wrapx(s, x);
  if (s->p.periodic_y) {
    y %= ly;
    if (y < 0) y += ly;
  } else {
    if (y < 0) return 1;
    if (y >= ly) return 2;
  }
  return s->solid[y * s->p.lx + x];
}

static double wall_temperature(const ora_state *s, int x, int y) {
  int fl = solid_at(s, x, y);
  return fl == 1 ? s->t_bottom[wrapx(s, x)] : s->p.t_top;
}

/* x-velocity of the solid cell in row y: the flat walls (ghost rows below
 * and above a non-periodic lattice) move with u_wall; solid cells inside
 * the lattice are at rest. */
static double wall_velocity(const ora_state *s, int y) {
  if (s->p.periodic_y) return 0.0;
  if (y < 0) return s->p.u_wall[0];
  if (y >= s->p.ly) return s->p.u_wall[1];
  return 0.0;
}

static int ora_default_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static double psi_exp(const ora_state *s, double rho) {
  return s->p.rho0 * (1.0 - exp(-rho / s->p.rho0));
}

/* Step 1: moments of the pre-collision populations at fluid nodes. */
static void moments(ora_state *s) {
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
  for (int k = 0; k < s->n; ++k) {
    double ra = 0, rb = 0, jx = 0, jy = 0, tt = 0;
    for (int i = 0; i < 9; ++i) {
      double a = s->f[0][i * s->n + k], b = s->f[1][i * s->n + k];
      ra += a;
      rb += b;
      jx += CX[i] * (a + b);
      jy += CY[i] * (a + b);
      tt += s->g[i * s->n + k];
    }
    s->rho[0][k] = ra;
    s->rho[1][k] = rb;
    s->jx[k] = jx;
    s->jy[k] = jy;
    s->temp[k] = tt;
  }
}

/* Step 2: pseudopotentials at every node, ghost rows included. Row index
 * yy = y + 2 of the padded grid. */
static void pseudopotentials(ora_state *s) {
  int lx = s->p.lx, ly = s->p.ly;
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
  for (int yy = 0; yy < ly + 4; ++yy) {
    int y = yy - 2;
    for (int x = 0; x < lx; ++x) {
      for (int l = 0; l < 2; ++l) {
        double r;
        if (solid_at(s, x, y)) {
          r = s->p.rho_wall[l];
        } else {
          int y0 = y;
          if (s->p.periodic_y) {
            y0 %= ly;
            if (y0 < 0) y0 += ly;
          }
          r = s->rho[l][y0 * lx + x];
        }
        s->psi_x[l][yy * lx + x] = r / s->p.rho0;
        s->psi_s[l][yy * lx + x] = psi_exp(s, r);
      }
    }
  }
}

static double padded(const ora_state *s, const double *a, int x, int y) {
  return a[(y + 2) * s->p.lx + wrapx(s, x)];
}

/* Step 3: forces on each component at fluid nodes. */
static void forces(ora_state *s) {
  int lx = s->p.lx, ly = s->p.ly;
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
  for (int y = 0; y < ly; ++y) {
    for (int x = 0; x < lx; ++x) {
      int k = y * lx + x;
      for (int l = 0; l < 2; ++l) {
        double fx = 0, fy = 0;
        if (!s->solid[k]) {
          int m = 1 - l;
          /* cross-component force, NN shell, psi = rho/rho0 (Eq. (7)) */
          double sx = 0, sy = 0;
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              double w = w_of(dx * dx + dy * dy);
              double v = padded(s, s->psi_x[m], x + dx, y + dy);
              sx += w * v * dx;
              sy += w * v * dy;
            }
          double px = padded(s, s->psi_x[l], x, y);
          fx += -s->p.g12 * px * sx;
          fy += -s->p.g12 * px * sy;
          /* short-range attraction, NN shell (Eq. (10)) */
          double ax = 0, ay = 0;
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              double w = w_of(dx * dx + dy * dy);
              double v = padded(s, s->psi_s[l], x + dx, y + dy);
              ax += w * v * dx;
              ay += w * v * dy;
            }
          double ps = padded(s, s->psi_s[l], x, y);
          fx += -s->p.g_a[l] * ps * ax;
          fy += -s->p.g_a[l] * ps * ay;
          /* mid-range repulsion, NN + NNN shells (Eq. (11)) */
          double rx = 0, ry = 0;
          for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
              double pw = p_of(dx * dx + dy * dy);
              double v = padded(s, s->psi_s[l], x + dx, y + dy);
              rx += pw * v * dx;
              ry += pw * v * dy;
            }
          fx += -s->p.g_r[l] * ps * rx;
          fy += -s->p.g_r[l] * ps * ry;
          /* buoyancy (Eq. (22)) */
          fy += s->rho[l][k] * s->p.alpha_g * s->temp[k];
        }
        s->fx[l][k] = fx;
        s->fy[l][k] = fy;
      }
    }
  }
}

/* Second-order equilibrium written as in Eq. (3): w_i rho [1 + u.c/cs2 +
 * u_k u_p (c_k c_p - cs2 delta_kp) / (2 cs2^2)]. */
static double equilibrium(int i, double rho, double ux, double uy) {
  double cu = CX[i] * ux + CY[i] * uy;
  double uu = ux * ux + uy * uy;
  return WGT[i] * rho * (1.0 + cu / CS2 + (cu * cu - CS2 * uu) / (2.0 * CS2 * CS2));
}

/* Hydrodynamic velocity u^H at fluid node k (needs moments and forces). */
static void hydro_velocity(const ora_state *s, int k, double *ux, double *uy) {
  double rho = s->rho[0][k] + s->rho[1][k];
  double fx = s->fx[0][k] + s->fx[1][k];
  double fy = s->fy[0][k] + s->fy[1][k];
  *ux = (s->jx[k] + 0.5 * fx) / rho;
  *uy = (s->jy[k] + 0.5 * fy) / rho;
}

/* Steps 4-5: velocities and BGK collision into fs, gs (fluid nodes only;
 * solid nodes get zeros). */
static void collide(ora_state *s) {
  double tau = s->p.tau, tau_g = s->p.tau_g;
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
  for (int k = 0; k < s->n; ++k) {
    if (s->solid[k]) {
      for (int i = 0; i < 9; ++i) {
        s->fs[0][i * s->n + k] = 0;
        s->fs[1][i * s->n + k] = 0;
        s->gs[i * s->n + k] = 0;
      }
      continue;
    }
    double rho = s->rho[0][k] + s->rho[1][k];
    double ux = s->jx[k] / rho, uy = s->jy[k] / rho;
    for (int l = 0; l < 2; ++l) {
      double rl = s->rho[l][k];
      double ulx = ux + tau * s->fx[l][k] / rl;
      double uly = uy + tau * s->fy[l][k] / rl;
      for (int i = 0; i < 9; ++i) {
        double f = s->f[l][i * s->n + k];
        s->fs[l][i * s->n + k] = f - (f - equilibrium(i, rl, ulx, uly)) / tau;
      }
    }
    double hx, hy;
    hydro_velocity(s, k, &hx, &hy);
    for (int i = 0; i < 9; ++i) {
      double g = s->g[i * s->n + k];
      s->gs[i * s->n + k] = g - (g - equilibrium(i, s->temp[k], hx, hy)) / tau_g;
    }
  }
}

/* Step 6: push streaming with bounce-back / anti-bounce-back at solid
 * targets. */
static void stream(ora_state *s) {
  int lx = s->p.lx, ly = s->p.ly, n = s->n;
  memset(s->fn[0], 0, sizeof(double) * 9 * n);
  memset(s->fn[1], 0, sizeof(double) * 9 * n);
  memset(s->gn, 0, sizeof(double) * 9 * n);
  /* every (target node, direction) pair is written exactly once */
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
  for (int y = 0; y < ly; ++y) {
    for (int x = 0; x < lx; ++x) {
      int k = y * lx + x;
      if (s->solid[k]) continue;
      for (int i = 0; i < 9; ++i) {
        int tx = x + CX[i], ty = y + CY[i];
        if (solid_at(s, tx, ty)) {
          int o = OPP[i];
          double uw = wall_velocity(s, ty);
          double cu = CX[i] * uw; /* c_i . u_w, c_i pointing into the wall */
          for (int l = 0; l < 2; ++l) {
            double rho_w = 0;
            for (int j = 0; j < 9; ++j) rho_w += s->fs[l][j * n + k];
            s->fn[l][o * n + k] = s->fs[l][i * n + k] - 2.0 * WGT[i] * rho_w * cu / CS2;
          }
          double even = 1.0 + cu * cu / (2.0 * CS2 * CS2) - uw * uw / (2.0 * CS2);
          s->gn[o * n + k] =
              -s->gs[i * n + k] + 2.0 * WGT[i] * wall_temperature(s, tx, ty) * even;
        } else {
          int txw = wrapx(s, tx), tyw = ty;
          if (s->p.periodic_y) {
            tyw %= ly;
            if (tyw < 0) tyw += ly;
          }
          int kt = tyw * lx + txw;
          s->fn[0][i * n + kt] = s->fs[0][i * n + k];
          s->fn[1][i * n + kt] = s->fs[1][i * n + k];
          s->gn[i * n + kt] = s->gs[i * n + k];
        }
      }
    }
  }
  double *tmp;
  for (int l = 0; l < 2; ++l) {
    tmp = s->f[l];
    s->f[l] = s->fn[l];
    s->fn[l] = tmp;
  }
  tmp = s->g;
  s->g = s->gn;
  s->gn = tmp;
}

static void macroscopic(ora_state *s) {
  moments(s);
  pseudopotentials(s);
  forces(s);
}

/* ------------------------------------------------------------------ API */

void ora_destroy(ora_state *s) {
  if (!s) return;
  for (int l = 0; l < 2; ++l) {
    free(s->f[l]); free(s->rho[l]); free(s->fx[l]); free(s->fy[l]);
    free(s->psi_s[l]); free(s->psi_x[l]); free(s->fs[l]); free(s->fn[l]);
  }
  free(s->g); free(s->solid); free(s->t_bottom); free(s->jx); free(s->jy);
  free(s->temp); free(s->gs); free(s->gn);
  free(s);
}

/* Build the state at t = 0: populations at the equilibria of the given
 * densities, temperature and (optional) velocity. Arrays are ly*lx with x
 * fastest; solid, ux0, uy0 may be NULL; t_bottom has lx entries. */
ora_state *ora_create(const ora_params *p, const double *rho_a,
                      const double *rho_b, const double *temp,
                      const double *ux0, const double *uy0,
                      const uint8_t *solid, const double *t_bottom) {
  if (!p || p->lx < 1 || p->ly < 1) return NULL;
  ora_state *s = (ora_state *)calloc(1, sizeof(ora_state));
  if (!s) return NULL;
  s->p = *p;
  s->nthreads = ora_default_threads();
  int n = p->lx * p->ly;
  s->n = n;
  size_t pad = (size_t)(p->ly + 4) * p->lx;
  int ok = 1;
  for (int l = 0; l < 2; ++l) {
    ok &= !!(s->f[l] = (double *)calloc(9 * (size_t)n, sizeof(double)));
    ok &= !!(s->fs[l] = (double *)calloc(9 * (size_t)n, sizeof(double)));
    ok &= !!(s->fn[l] = (double *)calloc(9 * (size_t)n, sizeof(double)));
    ok &= !!(s->rho[l] = (double *)calloc(n, sizeof(double)));
    ok &= !!(s->fx[l] = (double *)calloc(n, sizeof(double)));
    ok &= !!(s->fy[l] = (double *)calloc(n, sizeof(double)));
    ok &= !!(s->psi_s[l] = (double *)calloc(pad, sizeof(double)));
    ok &= !!(s->psi_x[l] = (double *)calloc(pad, sizeof(double)));
  }
  ok &= !!(s->g = (double *)calloc(9 * (size_t)n, sizeof(double)));
  ok &= !!(s->gs = (double *)calloc(9 * (size_t)n, sizeof(double)));
  ok &= !!(s->gn = (double *)calloc(9 * (size_t)n, sizeof(double)));
  ok &= !!(s->solid = (uint8_t *)calloc(n, 1));
  ok &= !!(s->t_bottom = (double *)calloc(p->lx, sizeof(double)));
  ok &= !!(s->jx = (double *)calloc(n, sizeof(double)));
  ok &= !!(s->jy = (double *)calloc(n, sizeof(double)));
  ok &= !!(s->temp = (double *)calloc(n, sizeof(double)));
  if (!ok) {
    ora_destroy(s);
    return NULL;
  }
  if (solid) memcpy(s->solid, solid, n);
  if (t_bottom) memcpy(s->t_bottom, t_bottom, sizeof(double) * p->lx);
  for (int k = 0; k < n; ++k) {
    if (s->solid[k]) continue;
    double ux = ux0 ? ux0[k] : 0.0, uy = uy0 ? uy0[k] : 0.0;
    for (int i = 0; i < 9; ++i) {
      s->f[0][i * n + k] = equilibrium(i, rho_a[k], ux, uy);
      s->f[1][i * n + k] = equilibrium(i, rho_b[k], ux, uy);
      s->g[i * n + k] = equilibrium(i, temp[k], ux, uy);
    }
  }
  return s;
}

/* Advance nsteps time steps. */
void ora_step(ora_state *s, int64_t nsteps) {
  for (int64_t it = 0; it < nsteps; ++it) {
    macroscopic(s);
    collide(s);
    stream(s);
    s->t += 1;
  }
}

int64_t ora_time(const ora_state *s) { return s->t; }

/* Fields at the current time: rho_a, rho_b, u^H (x, y), T. Solid cells
 * report the wall densities, zero velocity and the wall temperature. Any
 * output pointer may be NULL. */
void ora_fields(ora_state *s, double *rho_a, double *rho_b, double *ux,
                double *uy, double *temp) {
  macroscopic(s);
  int lx = s->p.lx;
  for (int k = 0; k < s->n; ++k) {
    double ra, rb, hx, hy, tt;
    if (s->solid[k]) {
      ra = s->p.rho_wall[0];
      rb = s->p.rho_wall[1];
      hx = hy = 0;
      tt = wall_temperature(s, k % lx, k / lx);
    } else {
      ra = s->rho[0][k];
      rb = s->rho[1][k];
      hydro_velocity(s, k, &hx, &hy);
      tt = s->temp[k];
    }
    if (rho_a) rho_a[k] = ra;
    if (rho_b) rho_b[k] = rb;
    if (ux) ux[k] = hx;
    if (uy) uy[k] = hy;
    if (temp) temp[k] = tt;
  }
}

/* Pre-collision populations f(t), g(t): three [9][ly][lx] arrays. */
void ora_populations(const ora_state *s, double *fa, double *fb, double *g) {
  size_t b = sizeof(double) * 9 * (size_t)s->n;
  if (fa) memcpy(fa, s->f[0], b);
  if (fb) memcpy(fb, s->f[1], b);
  if (g) memcpy(g, s->g, b);
}

/* Post-collision populations f*(t), g*(t) (before streaming); solid cells
 * hold zeros. */
void ora_post_collision(ora_state *s, double *fa, double *fb, double *g) {
  macroscopic(s);
  collide(s);
  size_t b = sizeof(double) * 9 * (size_t)s->n;
  if (fa) memcpy(fa, s->fs[0], b);
  if (fb) memcpy(fb, s->fs[1], b);
  if (g) memcpy(g, s->gs, b);
}

/* Observables at the current time, out[6] = {mass_a, mass_b, sum_T, Nu,
 * Nu_top, kinetic energy}; sums run over fluid nodes in row-major order. */
void ora_observables(ora_state *s, double *out) {
  macroscopic(s);
  int lx = s->p.lx, ly = s->p.ly;
  double kappa = CS2 * (s->p.tau_g - 0.5);
  double ma = 0, mb = 0, st = 0, uyt = 0, dyt = 0, ke = 0, top = 0;
  long nf = 0, ntop = 0;
  for (int y = 0; y < ly; ++y) {
    for (int x = 0; x < lx; ++x) {
      int k = y * lx + x;
      if (s->solid[k]) continue;
      double hx, hy;
      hydro_velocity(s, k, &hx, &hy);
      double tt = s->temp[k];
      double tn, ts;
      if (solid_at(s, x, y + 1))
        tn = 2.0 * wall_temperature(s, x, y + 1) - tt;
      else
        tn = s->temp[((y + 1) % ly) * lx + x];
      if (solid_at(s, x, y - 1))
        ts = 2.0 * wall_temperature(s, x, y - 1) - tt;
      else
        ts = s->temp[((y - 1 + ly) % ly) * lx + x];
      ma += s->rho[0][k];
      mb += s->rho[1][k];
      st += tt;
      uyt += hy * tt;
      dyt += 0.5 * (tn - ts);
      ke += hx * hx + hy * hy;
      nf += 1;
      if (y == ly - 1) {
        top += tt - s->p.t_top;
        ntop += 1;
      }
    }
  }
  double inv = nf ? 1.0 / (double)nf : 0.0;
  out[0] = ma;
  out[1] = mb;
  out[2] = st;
  out[3] = (uyt * inv - kappa * dyt * inv) / (kappa * s->p.dt_nominal / ly);
  out[4] = ntop ? 2.0 * ly / s->p.dt_nominal * (top / (double)ntop) : 0.0;
  out[5] = ke * inv;
}

/* xy stress at the current time (fluid nodes; zero at solid cells), two
 * [ly][lx] arrays, either may be NULL:
 *   sxy_visc  -(1 - 1/(2 tau)) sum_l sum_i c_ix c_iy (f_{l,i} - f^eq_i(rho_l, u_l))
 *   pxy_int   1/2 sum_l [ psi_s,l(x) sum_c (G^a_l w(c) + G^r_l p(c))
 *             psi_s,l(x+c) c_x c_y + G12 psi_x,l(x) sum_c w(c) psi_x,m(x+c)
 *             c_x c_y ]   (m the other component)
 * The total xy stress of the rheology is sxy_visc - pxy_int. */
void ora_stress(ora_state *s, double *sxy_visc, double *pxy_int) {
  macroscopic(s);
  int lx = s->p.lx, ly = s->p.ly, n = s->n;
  double tau = s->p.tau;
  for (int y = 0; y < ly; ++y) {
    for (int x = 0; x < lx; ++x) {
      int k = y * lx + x;
      double sv = 0, pi = 0;
      if (!s->solid[k]) {
        double rho = s->rho[0][k] + s->rho[1][k];
        double ux = s->jx[k] / rho, uy = s->jy[k] / rho;
        for (int l = 0; l < 2; ++l) {
          double rl = s->rho[l][k];
          double ulx = ux + tau * s->fx[l][k] / rl;
          double uly = uy + tau * s->fy[l][k] / rl;
          double neq = 0;
          for (int i = 0; i < 9; ++i)
            neq += CX[i] * CY[i] * (s->f[l][i * n + k] - equilibrium(i, rl, ulx, uly));
          sv += -(1.0 - 0.5 / tau) * neq;
          int m = 1 - l;
          double self = 0, cross = 0;
          for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
              int c2 = dx * dx + dy * dy;
              double gw = s->p.g_a[l] * w_of(c2) + s->p.g_r[l] * p_of(c2);
              self += gw * padded(s, s->psi_s[l], x + dx, y + dy) * dx * dy;
              cross += w_of(c2) * padded(s, s->psi_x[m], x + dx, y + dy) * dx * dy;
            }
          pi += 0.5 * padded(s, s->psi_s[l], x, y) * self;
          pi += 0.5 * s->p.g12 * padded(s, s->psi_x[l], x, y) * cross;
        }
      }
      if (sxy_visc) sxy_visc[k] = sv;
      if (pxy_int) pxy_int[k] = pi;
    }
  }
}

/* Droplets at the current time (Sec. 2.4 and Sec. 3.3.2 Eq. (25)).
 * A droplet is a 4-connected cluster of fluid nodes whose density of the
 * first component exceeds `threshold` (the bulk, rho_A > B_th), x periodic
 * (and y when the lattice is periodic in y). Droplets are numbered in the
 * order of their smallest node index k = y*lx + x (canonical labels). For
 * droplet i:
 *   root[i]   its smallest node index
 *   size[i]   number of nodes
 *   mass[i]   sum of rho_A over its nodes
 *   cx, cy    centre of mass sum rho_A X / sum rho_A, with each node's x
 *             taken within half a period of the root's x (wrapped back into
 *             [0, lx) at the end) and likewise y when periodic
 *   nu[i]     (u_y T - kappa dT/dy) / (kappa dt_nominal / ly) at the centre,
 *             u_y = u^H_y, dT/dy by central differences with the mirror
 *             value at solid neighbours (as in Nu), each field bilinearly
 *             interpolated between the four nodes around the centre (x
 *             periodic; y clamped to the lattice); solid nodes enter with
 *             u_y = 0, T = their wall temperature and dT/dy = 0
 * label (ly*lx, optional) receives the droplet number of each node, -1
 * outside droplets. At most cap droplets are written; returns the count. */
static double node_dTdy(const ora_state *s, int x, int y) {
  int lx = s->p.lx, ly = s->p.ly;
  int k = y * lx + x;
  if (s->solid[k]) return 0.0;
  double tt = s->temp[k], tn, ts;
  if (solid_at(s, x, y + 1)) tn = 2.0 * wall_temperature(s, x, y + 1) - tt;
  else tn = s->temp[((y + 1) % ly) * lx + x];
  if (solid_at(s, x, y - 1)) ts = 2.0 * wall_temperature(s, x, y - 1) - tt;
  else ts = s->temp[((y - 1 + ly) % ly) * lx + x];
  return 0.5 * (tn - ts);
}

static double bilinear(const double *f, int lx, int ly, int periodic_y, double x, double y) {
  if (!periodic_y) y = y < 0 ? 0 : (y > ly - 1 ? ly - 1 : y);
  int x0 = (int)floor(x), y0 = (int)floor(y);
  double ax = x - x0, ay = y - y0;
  int x1 = x0 + 1, y1 = y0 + 1;
  x0 = ((x0 % lx) + lx) % lx;
  x1 = ((x1 % lx) + lx) % lx;
  if (periodic_y) {
    y0 = ((y0 % ly) + ly) % ly;
    y1 = ((y1 % ly) + ly) % ly;
  } else if (y1 > ly - 1) {
    y1 = ly - 1;
  }
  return (1 - ax) * (1 - ay) * f[y0 * lx + x0] + ax * (1 - ay) * f[y0 * lx + x1] +
         (1 - ax) * ay * f[y1 * lx + x0] + ax * ay * f[y1 * lx + x1];
}

int64_t ora_droplets(ora_state *s, double threshold, int64_t cap, int64_t *root,
                     int64_t *size, double *mass, double *cx, double *cy, double *nu,
                     int32_t *label) {
  macroscopic(s);
  int lx = s->p.lx, ly = s->p.ly, n = s->n, per_y = s->p.periodic_y;
  int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int *queue = (int *)malloc(sizeof(int) * (size_t)n);
  double *uy = (double *)malloc(sizeof(double) * (size_t)n);
  double *dty = (double *)malloc(sizeof(double) * (size_t)n);
  double *tt = (double *)malloc(sizeof(double) * (size_t)n);
  if (!lab || !queue || !uy || !dty || !tt) {
    free(lab); free(queue); free(uy); free(dty); free(tt);
    return -1;
  }
  for (int k = 0; k < n; ++k) {
    double hx = 0, hy = 0;
    if (!s->solid[k]) hydro_velocity(s, k, &hx, &hy);
    uy[k] = hy;
    dty[k] = node_dTdy(s, k % lx, k / lx);
    tt[k] = s->solid[k] ? wall_temperature(s, k % lx, k / lx) : s->temp[k];
    lab[k] = -1;
  }
  double kappa = CS2 * (s->p.tau_g - 0.5);
  int64_t count = 0;
  /* flood fill from each unlabelled bulk node in increasing index order */
  for (int k0 = 0; k0 < n; ++k0) {
    if (lab[k0] >= 0 || s->solid[k0] || !(s->rho[0][k0] > threshold)) continue;
    int head = 0, tail = 0;
    queue[tail++] = k0;
    lab[k0] = (int32_t)count;
    int xr = k0 % lx, yr = k0 / lx;
    double m = 0, mx = 0, my = 0;
    int64_t sz = 0;
    while (head < tail) {
      int k = queue[head++];
      int x = k % lx, y = k / lx;
      double r = s->rho[0][k];
      double dx = x - xr, dy = y - yr;
      if (dx > 0.5 * lx) dx -= lx;
      if (dx < -0.5 * lx) dx += lx;
      if (per_y) {
        if (dy > 0.5 * ly) dy -= ly;
        if (dy < -0.5 * ly) dy += ly;
      }
      m += r;
      mx += r * (xr + dx);
      my += r * (yr + dy);
      sz += 1;
      const int nx[4] = {x + 1, x - 1, x, x};
      const int ny[4] = {y, y, y + 1, y - 1};
      for (int j = 0; j < 4; ++j) {
        int yy = ny[j];
        if (yy < 0 || yy >= ly) {
          if (!per_y) continue;
          yy = (yy + ly) % ly;
        }
        int kk = yy * lx + wrapx(s, nx[j]);
        if (lab[kk] >= 0 || s->solid[kk] || !(s->rho[0][kk] > threshold)) continue;
        lab[kk] = (int32_t)count;
        queue[tail++] = kk;
      }
    }
    if (count < cap) {
      double X = mx / m, Y = my / m;
      X = fmod(X, (double)lx);
      if (X < 0) X += lx;
      if (per_y) {
        Y = fmod(Y, (double)ly);
        if (Y < 0) Y += ly;
      }
      double u = bilinear(uy, lx, ly, per_y, X, Y);
      double t = bilinear(tt, lx, ly, per_y, X, Y);
      double g = bilinear(dty, lx, ly, per_y, X, Y);
      if (root) root[count] = k0;
      if (size) size[count] = sz;
      if (mass) mass[count] = m;
      if (cx) cx[count] = X;
      if (cy) cy[count] = Y;
      if (nu) nu[count] = (u * t - kappa * g) / (kappa * s->p.dt_nominal / ly);
    }
    count += 1;
  }
  if (label) memcpy(label, lab, sizeof(int32_t) * (size_t)n);
  free(lab); free(queue); free(uy); free(dty); free(tt);
  return count;
}

/* Replace the state by the streaming of the given post-collision
 * populations (three [9][ly][lx] arrays) and set the time to t: the state
 * becomes f(t) = stream(f*(t-1)). Used to check one step of another
 * implementation from its own post-collision state. */
void ora_load_post_collision(ora_state *s, const double *fa, const double *fb,
                             const double *g, int64_t t) {
  size_t b = sizeof(double) * 9 * (size_t)s->n;
  memcpy(s->fs[0], fa, b);
  memcpy(s->fs[1], fb, b);
  memcpy(s->gs, g, b);
  stream(s);
  s->t = t;
}

/* Threads of a state's parallel node loops (n >= 1). */
void ora_set_threads(ora_state *s, int n) { s->nthreads = n < 1 ? 1 : n; }
int ora_threads(const ora_state *s) { return s->nthreads; }
