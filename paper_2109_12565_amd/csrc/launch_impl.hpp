// Definitions of the launch interface, included once per storage type.
#pragma once

#include "launch.hpp"
#include "lb_kernels.hpp"
#include "lb_step2.hpp"

namespace tlbh {

namespace detail {

template <typename C>
tlbk::StepArgs<C> make_args(const Device& d, const void* src, void* dst) {
  tlbk::StepArgs<C> a{};
  const tlb_params& p = *d.p;
  a.src = src;
  a.dst = dst;
  a.link = d.link;
  a.solid = d.solid;
  a.t_bottom = static_cast<const C*>(d.t_bottom);
  a.partials = d.partials;
  a.fields = d.fields;
  a.lx = p.lx;
  a.ly = p.ly;
  a.pitch = d.pitch;
  a.rows_per_block = d.geo.rows;
  a.pop_stride = d.pop_stride;
  a.inv_tau = C(1.0 / p.tau);
  a.inv_tau_g = C(1.0 / p.tau_g);
  a.tau = C(p.tau);
  a.rho0 = C(p.rho0);
  a.inv_rho0 = C(1.0 / p.rho0);
  a.g12 = C(p.g12);
  a.ga0 = C(p.g_a[0]);
  a.ga1 = C(p.g_a[1]);
  a.gr0 = C(p.g_r[0]);
  a.gr1 = C(p.g_r[1]);
  a.alpha_g = C(p.alpha_g);
  a.t_top = C(p.t_top);
  a.rho_wall0 = C(p.rho_wall[0]);
  a.rho_wall1 = C(p.rho_wall[1]);
  a.ref_a = C(p.rho_ref[0]);
  a.ref_b = C(p.rho_ref[1]);
  a.ref_t = C(p.t_ref);
  a.uw0 = C(p.u_wall[0]);
  a.uw1 = C(p.u_wall[1]);
  return a;
}

template <class St, int BX, unsigned kMode>
void launch(const Device& d, const tlbk::StepArgs<typename St::C>& a) {
  hipLaunchKernelGGL((tlbk::lb_step_kernel<St, BX, kMode>), d.geo.grid, dim3(BX), 0, d.stream, a);
}

// Dispatch on offset width and block width (the 64-bit offset variant
// always runs 256-wide blocks).
template <class St, unsigned kMode>
void launch_geometry(const Device& d, const tlbk::StepArgs<typename St::C>& a) {
  if (d.geo.wide) launch<St, 256, kMode | tlbk::kModeWide>(d, a);
  else if (d.geo.bx == 256) launch<St, 256, kMode>(d, a);
  else launch<St, 64, kMode>(d, a);
}

// Dispatch on solid cells and on the tau = tau_g = 1 path (never for the
// stress pass, which needs the pulled populations themselves).
template <class St, unsigned kMode>
void launch_solid_tau(const Device& d, const tlbk::StepArgs<typename St::C>& a) {
  constexpr unsigned S = tlbk::kModeSolid, T1 = tlbk::kModeTauOne;
  if constexpr ((kMode & tlbk::kModeStress) != 0) {
    if (d.has_solid) launch_geometry<St, kMode | S>(d, a);
    else launch_geometry<St, kMode>(d, a);
  } else if (d.has_solid) {
    if (d.tau_one) launch_geometry<St, kMode | S | T1>(d, a);
    else launch_geometry<St, kMode | S>(d, a);
  } else {
    if (d.tau_one) launch_geometry<St, kMode | T1>(d, a);
    else launch_geometry<St, kMode>(d, a);
  }
}

// Dispatch on moving walls (a separate kernel, so walls at rest pay nothing
// for it; passes that read f(0) in place pull nothing and need no variant).
template <class St, unsigned kMode>
void launch_mode(const Device& d, const void* src, void* dst) {
  const auto a = make_args<typename St::C>(d, src, dst);
  if constexpr ((kMode & tlbk::kModeInit) == 0) {
    if (d.moving) {
      launch_solid_tau<St, kMode | tlbk::kModeMoving>(d, a);
      return;
    }
  }
  launch_solid_tau<St, kMode>(d, a);
}

template <class St, int BX, unsigned kMode>
int occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tlbk::lb_step_kernel<St, BX, kMode>, BX, 0) !=
          hipSuccess ||
      n < 1)
    n = 1;
  return n;
}

template <class St, unsigned kMode>
int occupancy_geometry(int bx, bool wide) {
  if (wide) return occupancy<St, 256, kMode | tlbk::kModeWide>();
  if (bx == 256) return occupancy<St, 256, kMode>();
  return occupancy<St, 64, kMode>();
}

template <class St, unsigned kMode>
void launch_step2_kernel(const Device& d, const tlbk::StepArgs<typename St::C>& a) {
  if (d.geo.lanes2 == kStep2LanesNarrow)
    hipLaunchKernelGGL((tlbk::lb_step2_kernel<St, kStep2LanesNarrow, kMode>), d.geo.grid2,
                       dim3(kStep2LanesNarrow), 0, d.stream, a, d.geo.strip2);
  else
    hipLaunchKernelGGL((tlbk::lb_step2_kernel<St, kStep2Lanes, kMode>), d.geo.grid2,
                       dim3(kStep2Lanes), 0, d.stream, a, d.geo.strip2);
}

// Storages with a two-step kernel: FP64, FP32 and the 16-bit floating
// deviations (FP32 rest planes); not the fixed-point one, whose exact
// mass needs every intermediate value on its grid.
template <class St>
constexpr bool kHasStep2 = !St::kFix && (!St::kDev || St::kRest32);

// Storages with the adjoint (FP64, FP32).
template <class St>
constexpr bool kHasAdjoint = !St::kFix && !St::kDev;

template <class St>
void launch_step2(const Device& d, const void* src, void* dst, Pass pass, void* moments) {
  if constexpr (kHasStep2<St>) {
    auto a = make_args<typename St::C>(d, src, dst);
    a.rows_per_block = d.geo.rows2;
    a.moments = moments;
    constexpr unsigned M = tlbk::kModeStore | tlbk::kModeTauOne;
    constexpr unsigned S = tlbk::kModeSolid, V = tlbk::kModeMoving;
    // the adjoint's variants: flat walls at rest only
    if (pass == Pass::kStep2TopRow) {
      if (!d.moving && !d.has_solid) launch_step2_kernel<St, M | tlbk::kModeTopRow>(d, a);
      return;
    }
    if (pass == Pass::kStep2Moments || pass == Pass::kStep2MomentsTopRow) {
      if constexpr (kHasAdjoint<St>) {
        constexpr unsigned MM = M | tlbk::kModeMoments;
        if (d.moving || d.has_solid) return;
        if (pass == Pass::kStep2Moments) launch_step2_kernel<St, MM>(d, a);
        else launch_step2_kernel<St, MM | tlbk::kModeTopRow>(d, a);
      }
      return;
    }
    if (d.moving) {
      if (d.has_solid) launch_step2_kernel<St, M | S | V>(d, a);
      else launch_step2_kernel<St, M | V>(d, a);
    } else {
      if (d.has_solid) launch_step2_kernel<St, M | S>(d, a);
      else launch_step2_kernel<St, M>(d, a);
    }
  }
}

template <class St, int BT, unsigned kMode>
int step2_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tlbk::lb_step2_kernel<St, BT, kMode>, BT,
                                                   0) != hipSuccess ||
      n < 1)
    n = 1;
  return n;
}

template <class St, unsigned kMode>
int step2_occupancy_lanes(int lanes) {
  return lanes == kStep2LanesNarrow ? step2_occupancy<St, kStep2LanesNarrow, kMode>()
                                    : step2_occupancy<St, kStep2Lanes, kMode>();
}

}  // namespace detail

template <class St>
int Launcher<St>::step2_blocks_per_cu(bool solid, int lanes) {
  if constexpr (detail::kHasStep2<St>) {
    constexpr unsigned M = tlbk::kModeStore | tlbk::kModeTauOne;
    return solid ? detail::step2_occupancy_lanes<St, M | tlbk::kModeSolid>(lanes)
                 : detail::step2_occupancy_lanes<St, M>(lanes);
  } else {
    (void)solid;
    (void)lanes;
    return 0;
  }
}

template <class St>
int Launcher<St>::blocks_per_cu(int bx, bool wide, bool solid, bool tau_one) {
  using namespace tlbk;
  constexpr unsigned S = kModeStore;
  if (solid) {
    return tau_one ? detail::occupancy_geometry<St, S | kModeSolid | kModeTauOne>(bx, wide)
                   : detail::occupancy_geometry<St, S | kModeSolid>(bx, wide);
  }
  return tau_one ? detail::occupancy_geometry<St, S | kModeTauOne>(bx, wide)
                 : detail::occupancy_geometry<St, S>(bx, wide);
}

template <class St>
void Launcher<St>::step(const Device& d, Pass pass, const void* src, void* dst, void* moments) {
  using namespace tlbk;
  switch (pass) {
    case Pass::kStep: detail::launch_mode<St, kModeStore>(d, src, dst); break;
    case Pass::kStepObserve: detail::launch_mode<St, kModeStore | kModeObserve>(d, src, dst); break;
    case Pass::kInitStep:
      detail::launch_mode<St, kModeStore | kModeInit | kModeObserve>(d, src, dst);
      break;
    case Pass::kObserve: detail::launch_mode<St, kModeObserve>(d, src, dst); break;
    case Pass::kObserveInit: detail::launch_mode<St, kModeObserve | kModeInit>(d, src, dst); break;
    case Pass::kFields: detail::launch_mode<St, kModeFields>(d, src, dst); break;
    case Pass::kFieldsInit: detail::launch_mode<St, kModeFields | kModeInit>(d, src, dst); break;
    case Pass::kStress: detail::launch_mode<St, kModeFields | kModeStress>(d, src, dst); break;
    case Pass::kStressInit:
      detail::launch_mode<St, kModeFields | kModeStress | kModeInit>(d, src, dst);
      break;
    case Pass::kStepMoments:
      if constexpr (detail::kHasAdjoint<St>) {
        if (d.tau_one && !d.moving && !d.has_solid) {
          auto a = detail::make_args<typename St::C>(d, src, dst);
          a.moments = moments;
          detail::launch_geometry<St, kModeStore | kModeTauOne | kModeMoments>(d, a);
        }
      }
      break;
    case Pass::kStep2:
    case Pass::kStep2TopRow:
    case Pass::kStep2Moments:
    case Pass::kStep2MomentsTopRow: detail::launch_step2<St>(d, src, dst, pass, moments); break;
  }
}

template <class St>
void Launcher<St>::init_equilibrium(const Device& d, void* buf, const double* rho_a,
                                    const double* rho_b, const double* temp, const double* ux0,
                                    const double* uy0) {
  using C = typename St::C;
  const tlb_params& p = *d.p;
  dim3 grid((p.lx + 255) / 256, p.ly, 1);
  hipLaunchKernelGGL(tlbk::lb_init_equilibrium<St>, grid, dim3(256), 0, d.stream,
                     static_cast<typename St::T*>(buf), rho_a, rho_b, temp, ux0, uy0, d.solid, p.lx,
                     p.ly, d.pitch, d.pop_stride, C(p.rho_ref[0]), C(p.rho_ref[1]), C(p.t_ref));
}

template <class St>
void Launcher<St>::export_populations(const Device& d, const void* buf, double* out) {
  using C = typename St::C;
  const tlb_params& p = *d.p;
  dim3 grid((p.lx + 255) / 256, p.ly, 27);
  hipLaunchKernelGGL(tlbk::lb_export_populations<St>, grid, dim3(256), 0, d.stream,
                     static_cast<const typename St::T*>(buf), out, d.solid, p.lx, p.ly, d.pitch,
                     d.pop_stride, C(p.rho_ref[0]), C(p.rho_ref[1]), C(p.t_ref));
}

}  // namespace tlbh
