// Launches of the discrete adjoint kernels (FP64 and FP32 storages).
#include "adjoint_kernels.hpp"
#include "launch.hpp"
#include "launch_impl.hpp"

namespace tlbh {

namespace {

template <class St>
tlbk::AdjArgs<typename St::C> adjoint_args(const Device& d, const AdjointWork& w,
                                           const void* state, int in) {
  using C = typename St::C;
  tlbk::AdjArgs<C> a{};
  a.s = detail::make_args<C>(d, state, nullptr);
  a.state = state;
  a.lam_next = static_cast<const C*>(w.lam[in]);
  a.lam = static_cast<C*>(w.lam[1 - in]);
  a.fbar = static_cast<C*>(w.fbar);
  a.Fbar = static_cast<C*>(w.Fbar);
  a.aux = static_cast<C*>(w.aux);
  a.rbar = static_cast<C*>(w.rbar);
  a.grad = w.grad;
  a.loss_terms = w.loss_terms;
  return a;
}

}  // namespace

template <class St>
void Adjoint<St>::top_row_term(const Device& d, const AdjointWork& w, const void* state, int k,
                               int stride) {
  auto a = adjoint_args<St>(d, w, state, 0);
  a.step_index = k;
  a.loss_stride = stride;
  hipLaunchKernelGGL((tlbk::adj_top_row_sum<St>), dim3(1), dim3(256), 0, d.stream, a);
}

template <class St>
void Adjoint<St>::reverse_step(const Device& d, const AdjointWork& w, const void* state, int in,
                               double kappa_top, const void* next_state, bool density_ready,
                               bool first) {
  using C = typename St::C;
  auto a = adjoint_args<St>(d, w, state, in);
  a.kappa_top = static_cast<C>(kappa_top);
  a.next_state = next_state;
  const int lx = d.p->lx, ly = d.p->ly;
  const dim3 grid((lx + 255) / 256, ly), block(256);
  // the stencil kernels run on 64 x 4 tiles
  const dim3 tiles((lx + tlbk::kAdjTX - 1) / tlbk::kAdjTX, (ly + tlbk::kAdjTY - 1) / tlbk::kAdjTY);
  if (d.tau_one) {
    // Two kernels per reverse step: adj_local gathers lambda(t+1) from the
    // previous step's compact planes, adj_scatter also does the T_b gradient
    // and the next step's densities. Buffers alternate by `in` (planes of
    // lambda[0], unused in this form): compact planes, dL/drho, densities.
    C* lam0 = static_cast<C*>(w.lam[0]);
    const size_t plane = (size_t)d.pop_stride;
    C* cmp[2] = {lam0, lam0 + 5 * plane};
    C* rb[2] = {lam0 + 10 * plane, lam0 + 12 * plane};
    C* aux[2] = {static_cast<C*>(w.aux), lam0 + 14 * plane};
    a.fbar = cmp[in];
    a.rbar = rb[in];
    a.aux = aux[in];
    a.cmp_prev = cmp[1 - in];
    a.rbar_prev = rb[1 - in];
    a.aux_next = aux[1 - in];
    a.have_prev = first ? 0 : 1;
    // state and next_state are moment-tape slots here
    a.mom = static_cast<const C*>(state);
    a.mom_next = static_cast<const C*>(next_state);
    a.state = nullptr;
    a.next_state = nullptr;
    if (!density_ready)
      hipLaunchKernelGGL((tlbk::adj_density_moments<St>), grid, block, 0, d.stream, a);
    hipLaunchKernelGGL((tlbk::adj_local<St, true>), tiles, block, 0, d.stream, a);
    hipLaunchKernelGGL((tlbk::adj_scatter<St, true>), tiles, block, 0, d.stream, a);
  } else {
    if (!density_ready) hipLaunchKernelGGL((tlbk::adj_density<St>), grid, block, 0, d.stream, a);
    hipLaunchKernelGGL((tlbk::adj_local<St, false>), tiles, block, 0, d.stream, a);
    hipLaunchKernelGGL((tlbk::adj_scatter<St, false>), tiles, block, 0, d.stream, a);
    hipLaunchKernelGGL((tlbk::adj_pull<St, false>), grid, block, 0, d.stream, a);
  }
}

template struct Adjoint<tlbk::Store<double>>;
template struct Adjoint<tlbk::Store<float>>;

}  // namespace tlbh
