// Host-side launch interface between the C ABI (tlb.hip) and the kernels.
// Each storage type's kernels are instantiated in a translation unit of their
// own (launch_<storage>.hip), compiled in parallel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tlb.h"

namespace tlbh {

struct Geometry {
  int bx = 64;       // columns (threads) per block
  int rows = 1;      // rows per block chunk
  bool wide = false; // 64-bit byte offsets (population buffer >= 4 GiB)
  dim3 grid;
  // fused two-step kernel (tau = tau_g = 1; flat walls at rest or moving);
  // rows2 == 0: not used
  int rows2 = 0;     // rows per block chunk
  int lanes2 = 256;  // lanes per block (kStep2Lanes or kStep2LanesNarrow)
  int strip2 = 0;    // stored columns per strip (lanes2 - kStep2Halo at most)
  dim3 grid2;
};

// Lanes per block of the two-step kernel (wide and narrow blocks) and the
// columns of each strip that only feed the others (5 on each side).
constexpr int kStep2Lanes = 256;
constexpr int kStep2LanesNarrow = 128;
constexpr int kStep2Halo = 10;

// Everything a launch needs from a handle.
struct Device {
  const tlb_params* p = nullptr;
  hipStream_t stream = nullptr;
  Geometry geo;
  int pitch = 0;
  long long pop_stride = 0;
  bool has_solid = false;
  bool tau_one = false;            // tau = tau_g = 1 path
  bool moving = false;             // a flat wall moves (u_wall != 0)
  const uint16_t* link = nullptr;
  const uint8_t* solid = nullptr;
  const void* t_bottom = nullptr;  // compute-type copy of the bottom temperature
  double* partials = nullptr;
  double* fields = nullptr;
};

// Kernel passes of the step kernel.
enum class Pass {
  kStep,         // f*(t) -> f*(t+1)
  kStepObserve,  // same, and the observable sums of time t+1 into partials
  kInitStep,     // f(0) in place -> f*(0), and the observable sums of t = 0
  kObserve,      // observable sums of time t from f*(t-1), no store
  kObserveInit,  // same at t = 0 from f(0)
  kFields,       // fields of time t from f*(t-1), no store
  kFieldsInit,   // same at t = 0 from f(0)
  kStress,       // fields and xy stress of time t (general path), no store
  kStressInit,   // same at t = 0 from f(0)
  kStep2,        // f*(t) -> f*(t+2), fused two-step kernel (Geometry::rows2 > 0)
  kStep2TopRow,  // same (flat walls at rest), and per strip the sums of T - t_top over
                 // the top row of both steps into Device::partials [2][strips]
  // The adjoint's tape at tau = 1 (flat walls at rest, FP64 / FP32): the
  // moments rho_A, rho_B, j_x, j_y, T of each step's pulled state, [5] planes
  // of pop_stride compute-type values per step.
  kStepMoments,         // kStep at tau = 1, and the step's moments
  kStep2Moments,        // kStep2, and the moments of both steps
  kStep2MomentsTopRow   // kStep2TopRow, and the moments of both steps
};

template <class St>
struct Launcher {
  // Resident blocks per CU of the step kernel for this geometry.
  static int blocks_per_cu(int bx, bool wide, bool solid, bool tau_one);
  // Resident blocks per CU of the two-step kernel; 0 where the storage has
  // no two-step kernel.
  static int step2_blocks_per_cu(bool solid, int lanes);
  // moments: the moment output of the kStep*Moments passes
  static void step(const Device& d, Pass pass, const void* src, void* dst,
                   void* moments = nullptr);
  // f(0) = equilibria of the initial fields (rho_a, rho_b, temp, ux0, uy0;
  // the velocities may be null).
  static void init_equilibrium(const Device& d, void* buf, const double* rho_a, const double* rho_b,
                               const double* temp, const double* ux0, const double* uy0);
  static void export_populations(const Device& d, const void* buf, double* out);
};

// Work buffers of the reverse sweep, in the compute type of the storage and
// the population layout (pitch, pop_stride).
struct AdjointWork {
  void* lam[2] = {nullptr, nullptr};  // adjoint populations, 27 planes each
  void* fbar = nullptr;               // dL/d(pulled populations), 27 planes
  void* Fbar = nullptr;               // dL/dF, 4 planes
  void* aux = nullptr;                // rho_A, rho_B, psi_A, psi_B, 4 planes
  void* rbar = nullptr;               // dL/drho from the force stencils, 2 planes
  double* grad = nullptr;             // [lx] dL/dT_b
  double* loss_terms = nullptr;       // [steps][stride] top-row sums of T - t_top (per
                                      // fused-kernel strip, or in slot 0)
};

// Number of compute-type planes of an AdjointWork.
constexpr int kAdjointPlanes = 27 * 2 + 27 + 4 + 4 + 2;

// Discrete adjoint of the flat-wall step, for the FP64 and FP32 storages.
template <class St>
struct Adjoint {
  // w.loss_terms[k] = sum over the top row of T - t_top, T the temperature
  // pulled from `state` (the step's pre-collision temperature).
  static void top_row_term(const Device& d, const AdjointWork& w, const void* state, int k,
                           int stride);
  // Reverse step of state -> next state: lambda[1 - in] from lambda[in]
  // (dL/d of the next state), adding the top-row loss term with weight
  // kappa_top and accumulating dL/dT_b into w.grad. density_ready: the
  // densities of `state` are already prepared (by the previous reverse
  // step); next_state (or null): the state of the following reverse step,
  // whose densities this step then prepares; first: the sweep's first
  // reverse step (lambda of the next state is zero). At tau = tau_g = 1 the
  // adjoint of a step is carried in compact per-node planes instead of
  // lambda, alternating with `in`, and `state` / `next_state` are the
  // moment-tape slots of the two steps (Pass::kStepMoments) instead of
  // states.
  static void reverse_step(const Device& d, const AdjointWork& w, const void* state, int in,
                           double kappa_top, const void* next_state, bool density_ready,
                           bool first);
};

}  // namespace tlbh
