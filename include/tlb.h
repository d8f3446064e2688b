/*
 * tlb.h - C ABI of the MI355X (gfx950) library for the thermal two-component
 * Shan-Chen lattice Boltzmann update of TLBfind (arXiv:2109.12565, Sec. 2).
 *
 * The library evolves, on one GPU, the 2D model of Sec. 2: two D2Q9 BGK fluid
 * components (Sec. 2.1 Eqs. (1)-(3)) coupled by the cross force (Eq. (7)) and
 * by self forces with short-range attraction (Eq. (10)) and mid-range
 * repulsion on a 25-point stencil (Eq. (11), weights of Fig. 1(b)); D2Q9
 * temperature populations (Sec. 2.3 Eqs. (16)-(18)) advected by the
 * hydrodynamic velocity and feeding back through Boussinesq buoyancy
 * (Eq. (22)); solid walls below and above the channel with wetting densities
 * (Sec. 2.2.1) and half-way bounce-back (Sec. 2.2), walls held at fixed
 * temperatures (Sec. 3.2.3); periodic x.
 *
 * Lattice and arrays. The lattice has lx columns (x, periodic) and ly rows
 * (y). Every host field array is ly*lx doubles, row-major with x fastest.
 * The wall planes lie half a cell below row 0 and half a cell above row
 * ly-1. Populations are indexed in this direction order (c_x, c_y):
 *   0 (0,0)  1 (1,0)  2 (0,1)  3 (-1,0)  4 (0,-1)
 *   5 (1,1)  6 (-1,1) 7 (-1,-1) 8 (1,-1)
 * and population arrays are [27][ly][lx]: f_A (0..8), f_B (9..17), g (18..26).
 *
 * Time. After tlb_init the state is at t = 0; tlb_step(n) advances to t + n.
 * Fields and observables at time t are the moments of the pre-collision
 * populations f(t) and the hydrodynamic velocity u^H(t) (Sec. 2.1: rho u^H =
 * rho u + F/2).
 *
 * Return codes: every function returns TLB_OK (0) or a negative code. No C++
 * exception crosses the ABI. The message of the last failure is returned by
 * tlb_last_error.
 *
 * Threading and streams: one handle is used by one host thread at a time.
 * All device work of a handle is enqueued on the stream given at init (or
 * on a stream the library creates); tlb_step only enqueues work, the calls
 * that return data to the host synchronise that stream.
 */
#ifndef TLB_H
#define TLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum tlb_status {
  TLB_OK = 0,
  TLB_EINVAL = -1,   /* bad argument: NULL pointer, size, tau <= 1/2, precision */
  TLB_ENOMEM = -2,   /* device or host allocation failed */
  TLB_EDEVICE = -3,  /* a HIP call failed (message in tlb_last_error) */
  TLB_ENUMERIC = -4, /* NaN or Inf in the FP64 mass reduction */
  TLB_ESTATE = -5    /* call not valid in the handle's current state */
};

/* Storage type of the populations in device memory. Collisions are computed
 * in FP64 for TLB_FP64 and in FP32 otherwise. The 16-bit forms store each
 * population as its deviation from a fixed reference: f_{l,i} - w_i
 * rho_ref[l] for the fluid components and g_i - w_i t_ref for the
 * temperature (halving the bytes moved per step).
 *   TLB_FP16_DEV, TLB_BF16_DEV: floating point, round to nearest even.
 *   TLB_FIX16_DEV: fixed point in units of 2^-15, deviations in [-1, 1)
 *     (saturating outside); the rest population takes the exact remainder
 *     of the stored sum, so each component's mass is conserved exactly. */
enum tlb_precision {
  TLB_FP64 = 0,
  TLB_FP32 = 1,
  TLB_FP16_DEV = 2,   /* IEEE binary16 deviations */
  TLB_BF16_DEV = 3,   /* bfloat16 deviations */
  TLB_FIX16_DEV = 4   /* 16-bit fixed-point deviations */
};

/* Kernel selection bits of tlb_params.launch_flags (0 for normal use; for
 * tests that compare the kernel variants and for tuning). */
enum tlb_launch_flags {
  TLB_LAUNCH_GENERAL_PATH = 1,  /* no tau = tau_g = 1 specialisation */
  TLB_LAUNCH_WIDE_OFFSETS = 2   /* 64-bit offsets even below 4 GiB */
};

/* tlb_params.fused: use of the fused two-step kernel (see tlb_step). */
enum tlb_fused_mode {
  TLB_FUSED_AUTO = 0,    /* where it pays (two blocks per CU: FP32, 16-bit) */
  TLB_FUSED_NEVER = 1,
  TLB_FUSED_ALWAYS = 2   /* wherever it applies */
};

/* Model constants (Sec. 2; values of Appendix A in parentheses) and launch
 * choices (zero: chosen by the library). */
typedef struct tlb_params {
  int32_t lx, ly;        /* lattice size: lx >= 1, ly >= 1 */
  int32_t precision;     /* enum tlb_precision */
  int32_t launch_flags;  /* enum tlb_launch_flags bits, normally 0 */
  double tau;            /* fluid relaxation time, > 1/2 (1.0) */
  double tau_g;          /* thermal relaxation time, > 1/2 (1.0) */
  double rho0;           /* pseudopotential reference density, > 0 (0.83) */
  double g12;            /* cross coupling G_12 of Eq. (7) (0.405) */
  double g_a[2];         /* attraction G^a_11, G^a_22 of Eq. (10) (-9.0, -8.0) */
  double g_r[2];         /* repulsion G^r_11, G^r_22 of Eq. (11) (8.1, 7.1) */
  double alpha_g;        /* buoyancy alpha*g of Eq. (22) */
  double t_top;          /* top wall temperature */
  double rho_wall[2];    /* wetting densities of both components at solid
                            nodes (Sec. 2.2.1) (0.612, 0.612) */
  double dt_nominal;     /* Delta T in the Nusselt normalisation, != 0 */
  double rho_ref[2];     /* reference densities of the 16-bit storages */
  double t_ref;          /* reference temperature of the 16-bit storages */
  double u_wall[2];      /* x-velocity of the bottom and top walls (Couette
                            walls, Sec. 2.2 and Sec. 3.2.2); 0 for walls at
                            rest. A link into a moving wall is bounced back
                            with the momentum term 6 w_i rho c_ix u_w (rho the
                            boundary node's own density) and g against
                            2 w_i T_w (1 + 4.5 (c_i.u_w)^2 - 1.5 u_w^2);
                            solid cells inside the lattice do not move */
  int32_t fused;         /* enum tlb_fused_mode */
  int32_t fused_rows;    /* rows per chunk of the fused kernel (1..4096), 0: chosen */
  int32_t fused_strip;   /* at most this many stored columns per fused strip
                            (1..245), 0: chosen */
  int32_t rows;          /* rows per chunk of the single-step kernel (1..4096),
                            0: chosen */
  int32_t fused_lanes;   /* lanes per block of the fused kernel, 128 or 256
                            (at most lanes - 10 stored columns per strip),
                            0: chosen */
} tlb_params;

/* Observables at time `step` (Sec. 3.1, Sec. 3.3.2 Eq. (24)); sums and means
 * run over fluid nodes and are accumulated in FP64:
 *   mass_a, mass_b  sum of rho_A, rho_B
 *   sum_t           sum of T
 *   nu              (<u^H_y T> - kappa <dT/dy>) / (kappa dt_nominal / ly),
 *                   kappa = (tau_g - 1/2)/3, dT/dy by central differences
 *                   with the mirror value 2 T_w - T at a solid neighbour
 *   nu_top          2 ly / dt_nominal * mean over fluid nodes of row ly-1 of
 *                   (T - t_top): the top-wall heat flux in Nusselt units
 *   ke              mean of |u^H|^2 */
typedef struct tlb_obs {
  int64_t step;
  double mass_a, mass_b, sum_t, nu, nu_top, ke;
} tlb_obs;

/* One droplet (Sec. 2.4; droplet Nusselt number of Sec. 3.3.2 Eq. (25)). */
typedef struct tlb_droplet {
  int64_t root;   /* smallest node index y*lx + x of the droplet */
  int64_t size;   /* number of nodes */
  double mass;    /* sum of rho_A over its nodes */
  double x, y;    /* centre of mass (x in [0, lx)) */
  double nu;      /* droplet Nusselt number at the centre */
} tlb_droplet;

typedef struct tlb_handle tlb_handle;

/* Create a handle and set the state at t = 0 to the equilibria of the given
 * densities, temperature and velocity (Sec. 2.1 Eq. (3), Sec. 2.3 Eq. (18)).
 *   out        receives the handle (set to NULL on failure)
 *   p          model constants (copied)
 *   rho_a, rho_b, temp   host, ly*lx: initial densities and temperature
 *   ux0, uy0   host, ly*lx, or NULL for a fluid at rest
 *   solid      host, ly*lx, or NULL for flat walls only: 0 fluid node,
 *              1 solid node held at the bottom temperature of its column,
 *              2 solid node held at t_top
 *   t_bottom   host, lx: bottom wall temperature per column
 *   hip_stream hipStream_t to run on, or NULL for a library-owned stream
 * Host arrays are read during the call only. Device memory is owned by the
 * handle until tlb_destroy. Errors: TLB_EINVAL, TLB_ENOMEM, TLB_EDEVICE. */
int tlb_init(tlb_handle **out, const tlb_params *p, const double *rho_a,
             const double *rho_b, const double *temp, const double *ux0,
             const double *uy0, const uint8_t *solid, const double *t_bottom,
             void *hip_stream);

/* Device bytes of the workspace tlb_init_external needs for these
 * parameters and solid flags (host, ly*lx, or NULL): both population
 * buffers, the per-block observable partials, the observables, the bottom
 * temperature, the solid flags and the link masks, each part 256-byte
 * aligned. Queries the current device (the launch geometry depends on it).
 * Returns the byte count, or TLB_EINVAL for invalid parameters. */
int64_t tlb_workspace_bytes(const tlb_params *p, const uint8_t *solid);

/* tlb_init with the step path's device buffers placed in a caller's device
 * allocation on the current device (`workspace`, workspace_bytes >=
 * tlb_workspace_bytes(p, solid), 256-byte aligned), for callers whose
 * framework owns device memory (a PyTorch tensor, say). The caller keeps
 * the workspace alive and does not touch it until tlb_destroy, which does
 * not free it. Analyses (fields, stress, droplets, the adjoint's tape) still
 * allocate their own buffers on first use. Errors as tlb_init, and
 * TLB_EINVAL for a NULL, misaligned or too small workspace. */
int tlb_init_external(tlb_handle **out, const tlb_params *p, const double *rho_a,
                      const double *rho_b, const double *temp, const double *ux0,
                      const double *uy0, const uint8_t *solid, const double *t_bottom,
                      void *hip_stream, void *workspace, int64_t workspace_bytes);

/* Advance nsteps >= 0 time steps of Eqs. (1) and (16): per node, pull
 * streaming with bounce-back / anti-bounce-back at solid links, moments,
 * forces, velocity shift (Eq. (6)) and BGK collision. Enqueues only. With
 * tau = tau_g = 1 (the collision then returns the equilibria of Eqs. (3),
 * (18)), pairs of steps may run as one fused launch where the handle's
 * storage and lattice allow it (see tlb_launch_info; flat walls at rest or
 * moving, posts allowed); the last step of a call is always a single step,
 * which also forms the observable sums of the new time, and results agree
 * with single steps to rounding. Returns TLB_EINVAL for nsteps < 0 or a
 * NULL handle, TLB_EDEVICE on a launch failure. */
int tlb_step(tlb_handle *h, int64_t nsteps);

/* Observables at the current time (synchronises the stream). After
 * tlb_init and tlb_step the sums are already on the device (formed by the
 * last step); after a taped run or a new bottom temperature the time level
 * is evaluated again. Returns TLB_ENUMERIC if a component mass is not
 * finite. */
int tlb_observables(tlb_handle *h, tlb_obs *out);

/* Fields at the current time into host arrays of ly*lx doubles (any may be
 * NULL): densities, hydrodynamic velocity u^H and temperature. Solid nodes
 * report the wall densities, zero velocity and their wall temperature.
 * Synchronises the stream. */
int tlb_get_fields(tlb_handle *h, double *rho_a, double *rho_b, double *ux,
                   double *uy, double *temp);

/* xy stress at the current time into host arrays of ly*lx doubles (either
 * may be NULL; zero at solid nodes). The total stress of the rheology
 * (Sec. 2.1 below Eq. (14), Sec. 3.2.2) is sxy_visc - pxy_int:
 *   sxy_visc  viscous part -(1 - 1/(2 tau)) sum_l sum_i c_ix c_iy
 *             (f_{l,i} - f^eq_i(rho_l, u_l)) of the pre-collision f(t)
 *   pxy_int   xy component of the interaction pressure tensor of the forces
 *             of Eqs. (7), (10), (11): 1/2 sum_l [psi_l(x) sum_c (G^a_l w(c)
 *             + G^r_l p(c)) psi_l(x+c) c_x c_y + G12 (rho_l(x)/rho0)
 *             sum_c w(c) (rho_m(x+c)/rho0) c_x c_y], m the other component
 * Synchronises the stream. */
int tlb_get_stress(tlb_handle *h, double *sxy_visc, double *pxy_int);

/* Row averages over the fluid nodes of each row at the current time (the
 * x-averaged profiles of the Couette rheology, Sec. 3.2.2): u_av[y] = mean
 * of u^H_x, pxy_av[y] = mean of sxy_visc - pxy_int (see tlb_get_stress).
 * Host arrays of ly doubles, either may be NULL; rows without fluid report
 * 0. Deterministic (fixed-order FP64 sums). Synchronises the stream. */
int tlb_row_averages(tlb_handle *h, double *u_av, double *pxy_av);

/* Droplets at the current time. A droplet is a 4-connected cluster of fluid
 * nodes whose rho_A exceeds `threshold` (the bulk, B_th = 0.8 in the paper's
 * runs), x periodic; droplets are numbered in the order of their smallest
 * node index (independent of scheduling). For each: its size, mass sum
 * rho_A, centre of mass (each node's x taken within half a period of the
 * smallest node's x, the result wrapped into [0, lx)), and the droplet
 * Nusselt number (u_y T - kappa dT/dy) / (kappa dt_nominal / ly) with u^H_y,
 * T and dT/dy (central differences, mirror value at solid neighbours; solid
 * nodes enter with u = 0, their wall temperature and dT/dy = 0) bilinearly
 * interpolated at the centre (x periodic, y clamped to [0, ly-1]).
 *   out     host array of cap entries (may be NULL if cap == 0)
 *   count   receives the number of droplets (may exceed cap: only the first
 *           cap are written)
 *   labels  host, ly*lx, or NULL: droplet number of each node, -1 outside
 * Sums are exact (fixed point, order independent). Synchronises the stream.
 * Errors: TLB_EINVAL, TLB_ENOMEM, TLB_EDEVICE. */
int tlb_droplets(tlb_handle *h, double threshold, tlb_droplet *out, int64_t cap,
                 int64_t *count, int32_t *labels);

/* tlb_droplets for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same results, computed in a static workspace that the library holds
 * on each device from its first tlb_init there until the process ends
 * (about 28 MiB), with no allocation or free of any kind. Limits: at most
 * 2^19 lattice nodes, 8192 columns and 16384 droplets; a larger lattice is
 * rejected with TLB_EINVAL before any work, more droplets with TLB_EINVAL
 * after the count (which is still returned). All handles on one device
 * share the workspace and each call overwrites it: calls that overlap in
 * time on one device (other threads or streams) race and must be
 * serialised by the caller. Synchronises the stream. Errors: TLB_EINVAL,
 * TLB_EDEVICE. */
int tlb_droplets_noalloc(tlb_handle *h, double threshold, tlb_droplet *out, int64_t cap,
                         int64_t *count, int32_t *labels);

/* Post-collision populations f*(t) of the current time (the state the next
 * step streams) as host doubles [27][ly][lx]; zero at solid nodes.
 * Synchronises the stream. */
int tlb_get_populations(tlb_handle *h, double *out);

/* Replace the bottom wall temperature (host, lx values); takes effect for
 * the following steps and observable evaluations. */
int tlb_set_bottom_temperature(tlb_handle *h, const double *t_bottom);

/* Taped forward run for the discrete adjoint (flat walls only, FP64 or FP32
 * storage). Advances nsteps >= 1 steps exactly as tlb_step does, keeping a
 * device copy of the state f* every ckpt_every >= 1 steps (the first at the
 * current time t0; ckpt_every = 0: 1 when the tape of every step fits in
 * half of the free device memory, else the shortest interval whose
 * checkpoints do), and evaluates the loss
 *   L = (1/nsteps) sum_{t = t0+1}^{t0+nsteps} Nu_top(t),
 * Nu_top(t) = 2 ly / dt_nominal * mean over row ly-1 of (T(t) - t_top), the
 * time-averaged top-wall Nusselt number (Sec. 3.3.2, Eq. (24) in top-wall
 * flux form), as a function of the bottom wall temperature T_b.
 *   loss  host, receives L (may be NULL)
 * The tape (checkpoints) replaces any previous one and stays valid until the
 * next tlb_forward_taped, tlb_set_bottom_temperature or tlb_destroy; later
 * tlb_step calls do not touch it. Checkpoint memory is
 * ceil(nsteps / ckpt_every) copies of the state. ckpt_every = 1 keeps every
 * step instead and the reverse sweep recomputes nothing: at tau = tau_g = 1
 * the steps write the moments rho_A, rho_B, j, T of their pulled state (5
 * values per node; the adjoint of a step at tau = 1 needs nothing else) and
 * no state is kept, otherwise every state. Synchronises the stream.
 * Errors: TLB_EINVAL (solid cells, moving walls, 16-bit storage, bad counts,
 * state buffer of 4 GiB or more, lx < 3, ly > 65535), TLB_ENOMEM,
 * TLB_EDEVICE. */
int tlb_forward_taped(tlb_handle *h, int64_t nsteps, int32_t ckpt_every, double *loss);

/* Reverse sweep of the taped run: grad_t_bottom (host, lx doubles) receives
 * seed * dL/dT_b(x), the exact derivative of the discrete forward map (the
 * adjoint of Eqs. (1)-(3), (6)-(12), (16)-(18), (22) and of the
 * anti-bounce-back wall source 2 w_i T_b). Each checkpoint segment is
 * recomputed (at tau = tau_g = 1 into the moments of its ckpt_every steps,
 * on a second stream the handle owns, one segment ahead of the sweep and
 * ordered with the handle's stream by events; else into ckpt_every - 1
 * states; nothing for ckpt_every = 1), then swept backwards one step at a
 * time. nsteps must equal the taped count. The
 * handle's current state is not changed. Synchronises the stream.
 * Errors: TLB_ESTATE (no valid tape, or nsteps differs from it),
 * TLB_EINVAL (NULL grad_t_bottom), TLB_ENOMEM, TLB_EDEVICE. */
int tlb_adjoint_step(tlb_handle *h, int64_t nsteps, double seed, double *grad_t_bottom);

/* Current time step. Returns -1 for a NULL handle. */
int64_t tlb_time(const tlb_handle *h);

/* Launch geometry chosen by tlb_init for the step kernels (Sec. 2.5 maps the
 * lattice onto GPU threads; here a block of `bx` threads marches over a
 * chunk of `rows` rows of a `bx`-column strip). fused_rows > 0 means that
 * tlb_step advances pairs of steps with the fused two-step kernel (tau =
 * tau_g = 1, flat walls at rest or moving; blocks of fused_lanes lanes,
 * strips of fused_strip stored columns, chunks of fused_rows rows); every
 * tlb_step call still ends with a single step. Host struct, written by the
 * call. Returns TLB_EINVAL on a NULL argument. */
typedef struct tlb_launch {
  int32_t bx, rows, grid_x, grid_y;
  int32_t fused_rows, fused_strip, fused_grid_x, fused_grid_y;
  int32_t fused_lanes;
} tlb_launch;
int tlb_launch_info(const tlb_handle *h, tlb_launch *out);

/* Free the handle and its device memory. NULL is accepted. */
int tlb_destroy(tlb_handle *h);

/* Message of the last failure on h (or of the calling thread's last failed
 * tlb_init when h is NULL); empty string if none. Valid until the next call
 * on the same handle. */
const char *tlb_last_error(const tlb_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* TLB_H */
