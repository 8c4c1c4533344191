// Plasma particle kernels (gfx950): field gather, fifth-order Adams-Bashforth
// push in zeta and charge/current deposition, fused in one pass over the
// particle slice (HiPACE++, arXiv:2109.10277, Sec. III.B), plus plasma
// initialisation and state import/export.  The per-tile body lives in
// push_tile.hpp.
#include "common.hpp"
#include "kernels.hpp"
#include "partials.hpp"
#include "push_tile.hpp"
#include "beam_body.hpp"

namespace qsp {

using push_detail::push_tile;
using push_detail::tile_shape;
using push_detail::TileShape;

// Waves per SIMD the compiler keeps room for: the FP32 linear-shape real
// push is held to five (its histogram tiles already allow five workgroups
// per CU), the FP32 linear-shape later trial push to eight (all 2048 tiles
// of a 1024^2 lattice resident at once); the other instances take what
// their registers allow.
template <typename T, int MODE, int O>
constexpr int push_waves() {
  if (sizeof(T) != 4 || O != 1) return 1;
  return MODE == kPushReal ? 5 : MODE == kTrialLater ? 8 : 1;
}

template <typename T, int MODE, int O>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(push_waves<T, MODE, O>())))
k_push(Geom g, Lattice L, PushArgs<T> a, DevCounters* ctr) {
  const bool first = blockIdx.x == 0 && blockIdx.y == 0;
  if (MODE == kPushTrial || MODE == kPushTrialTape || MODE == kTrialLater) {
    if (ctr->pc_done) return;
    // convergence of the previous corrector solve of this slice
    if (a.pc_partial && a.pc_iter > 0 &&
        partials::pc_consume(a.pc_partial, a.pc_nblk, a.pc_tol, ctr, first))
      return;
  }
  if (MODE == kPushReal && first && a.pc_partial && !ctr->pc_done)
    partials::pc_consume(a.pc_partial, a.pc_nblk, a.pc_tol, ctr, true);   // the last solve
  if (MODE == kPushReal && first && threadIdx.x == 0) {
    // close the slice's predictor-corrector bookkeeping
    const double r = ctr->pc_resid;
    if (a.iters_out) *a.iters_out = static_cast<int32_t>(ctr->pc_iters);
    if (a.iters_own) *a.iters_own = static_cast<int32_t>(ctr->pc_iters);
    if (a.resid_out) *a.resid_out = r;
    if (r > ctr->max_resid || r != r) ctr->max_resid = r;
    if (a.pc_tol > 0.0 && !ctr->pc_done) {
      if (static_cast<int>(ctr->pc_iters) >= a.pc_max_iter) ctr->pc_not_converged += 1ull;
      else if (a.pc_budgeted) ctr->budget_short += 1u;
    }
  }
  if constexpr (MODE == kPushReal) {
    // beam work riding on the launch: grid rows beyond the lattice tiles
    const int nty = L.nY / tile_shape(L, a.tile_rows, a.tile_halo).ty;
    if (static_cast<int>(blockIdx.y) >= nty) {
      const BeamRide& br = a.beam;
      const int b = (static_cast<int>(blockIdx.y) - nty) * static_cast<int>(gridDim.x) +
                    static_cast<int>(blockIdx.x);
      if (b < br.push_wgs)
        beam_detail::beam_push_range<T, O>(g, br.soa, br.n, br.off, a.k, a.f, br.dt,
                                           static_cast<int64_t>(b) * kBlock + threadIdx.x,
                                           static_cast<int64_t>(br.push_wgs) * kBlock);
      else if (b < br.push_wgs + br.dep_wgs)
        beam_detail::beam_deposit_range<O>(
            g, br.soa, br.n, br.off, a.k + 1, a.dzeta, a.dep.ch[0], a.dep.ch[3], nullptr,
            static_cast<int64_t>(b - br.push_wgs) * kBlock + threadIdx.x,
            static_cast<int64_t>(br.dep_wgs) * kBlock);
      return;
    }
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if constexpr (MODE == kExplicitDep)
    push_detail::explicit_tile<T, O>(g, L, a, blockIdx.x, blockIdx.y,
                                     reinterpret_cast<double*>(smem_raw));
  else if constexpr (MODE == kPushTrialTape)
    push_tile<T, kPushTrial, O, true>(g, L, a, ctr, blockIdx.x, blockIdx.y,
                                      reinterpret_cast<double*>(smem_raw));
  else
    push_tile<T, MODE, O>(g, L, a, ctr, blockIdx.x, blockIdx.y,
                          reinterpret_cast<double*>(smem_raw));
}

template <typename T>
__global__ void k_init_plasma(Lattice L, Particles<T> p, T w0) {
  const size_t np = static_cast<size_t>(L.np);
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < np;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    p.xi_x[i] = T(0);
    p.xi_y[i] = T(0);
    p.ux[i] = T(0);
    p.uy[i] = T(0);
    p.psi[i] = T(0);
    p.w[i] = w0;
#pragma unroll
    for (int c = 0; c < 20; ++c) p.hist[c * np + i] = T(0);
#pragma unroll
    for (int c = 0; c < 5; ++c) p.pab[c * np + i] = T(0);
  }
}

template <typename T>
__global__ void k_import_state(Geom g, Lattice L, Particles<T> p, const double* x,
                               const double* y, const double* ux, const double* uy,
                               const double* psi, const double* w, const double* hist, int k,
                               double dzeta) {
  const size_t np = static_cast<size_t>(L.np);
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < np;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int I = static_cast<int>(i % L.nX), J = static_cast<int>(i / L.nX);
    const double sx = (I + 0.5) / L.ppc_x, sy = (J + 0.5) / L.ppc_y;
    p.xi_x[i] = static_cast<T>((x[i] - g.x_lo) / g.hx - sx);
    p.xi_y[i] = static_cast<T>((y[i] - g.y_lo) / g.hy - sy);
    p.ux[i] = static_cast<T>(ux[i]);
    p.uy[i] = static_cast<T>(uy[i]);
    p.psi[i] = static_cast<T>(psi[i]);
    p.w[i] = static_cast<T>(w[i]);
    T hv[4][5];
    for (int m = 0; m < 4; ++m) {
      const int slot = (k - 1 - m + 8) & 3;
      for (int c = 0; c < 5; ++c) {
        double v = hist[(m * 5 + c) * np + i];
        if (c == 0) v /= g.hx;
        if (c == 1) v /= g.hy;
        hv[m][c] = static_cast<T>(v);
        p.hist[(slot * 5 + c) * np + i] = hv[m][c];
      }
    }
    const T y[5] = {p.xi_x[i], p.xi_y[i], p.ux[i], p.uy[i], p.psi[i]};
    const T dz = static_cast<T>(dzeta);
    for (int c = 0; c < 5; ++c)
      p.pab[c * np + i] = ab5_history(y[c], hv[0][c], hv[1][c], hv[2][c], hv[3][c], dz);
  }
}

template <typename T>
__global__ void k_export_state(Geom g, Lattice L, Particles<T> p, double* x, double* y,
                               double* ux, double* uy, double* psi, double* w, double* hist,
                               int k) {
  const size_t np = static_cast<size_t>(L.np);
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < np;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int I = static_cast<int>(i % L.nX), J = static_cast<int>(i / L.nX);
    const double sx = (I + 0.5) / L.ppc_x, sy = (J + 0.5) / L.ppc_y;
    x[i] = g.x_lo + (sx + static_cast<double>(p.xi_x[i])) * g.hx;
    y[i] = g.y_lo + (sy + static_cast<double>(p.xi_y[i])) * g.hy;
    ux[i] = p.ux[i];
    uy[i] = p.uy[i];
    psi[i] = p.psi[i];
    w[i] = p.w[i];
    for (int m = 0; m < 4; ++m) {
      const int slot = (k - 1 - m + 8) & 3;
      for (int c = 0; c < 5; ++c) {
        double v = p.hist[(slot * 5 + c) * np + i];
        if (c == 0) v *= g.hx;
        if (c == 1) v *= g.hy;
        hist[(m * 5 + c) * np + i] = v;
      }
    }
  }
}

// ------------------------------------------------------------------ launchers
static dim3 grid_1d(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 65536) b = 65536;
  if (b == 0) b = 1;
  return dim3(static_cast<unsigned>(b));
}

template <typename T>
void launch_init_plasma(const Lattice& L, const Particles<T>& p, double w0, hipStream_t st) {
  hipLaunchKernelGGL(k_init_plasma<T>, grid_1d(L.np), dim3(kBlock), 0, st, L, p,
                     static_cast<T>(w0));
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_push(const Geom& g, const Lattice& L, const PushArgs<T>& a, PushMode mode,
                 DevCounters* ctr, hipStream_t st) {
  const TileShape ts = tile_shape(L, a.tile_rows, a.tile_halo);
  const bool trial = mode == kPushTrial || mode == kPushTrialTape || mode == kTrialLater;
  const int nch = trial ? 2 : (mode == kExplicitDep ? 3 : 4);
  const size_t lds = a.tiled ? static_cast<size_t>(nch) * ts.nw * ts.nh * sizeof(double) : 0;
  if (lds > 160 * 1024) throw std::invalid_argument("push tile histogram exceeds the LDS");
  // a real push carries beam workgroups in extra grid rows
  const int extra = mode == kPushReal ? a.beam.push_wgs + a.beam.dep_wgs : 0;
  if (a.beam.push_wgs < 0 || a.beam.dep_wgs < 0 ||
      (extra > 0 && (!a.beam.soa || !a.beam.off || a.beam.n <= 0)))
    throw std::invalid_argument("beam work of a real push: bad arguments");
  const int ntx = L.nX / ts.tx;
  const dim3 grid(ntx, L.nY / ts.ty + (extra + ntx - 1) / ntx);
  // the later trial push and the gathers address a particle or field plane
  // with 32-bit byte offsets
  if (static_cast<uint64_t>(L.np) * sizeof(T) >= (1ull << 32) ||
      static_cast<uint64_t>(g.nx) * g.ny * sizeof(T) >= (1ull << 32))
    throw std::invalid_argument("a particle or field plane of 4 GiB or more");
  // an owner flush writes every node once only if the tiles cover the lattice
  if (L.nX % ts.tx || L.nY % ts.ty)
    throw std::invalid_argument("push tiles must divide the particle lattice");
  if (a.dep.sh[0] && !trial)
    throw std::invalid_argument("shared deposit planes are for the trial pushes");
  if (mode == kTrialLater && !a.rec)
    throw std::invalid_argument("a later trial push needs the first one's record");
  if (mode == kPushTrialTape && !a.tape)
    throw std::invalid_argument("a taped trial push needs the tape's particle planes");
  if (mode == kExplicitDep && g.order < 1)
    throw std::invalid_argument("the explicit Bx/By solver needs a shape order of 1, 2 or 3");
  auto run = [&](auto order) {
    constexpr int O = decltype(order)::value;
    constexpr int OE = O < 1 ? 1 : O;   // the explicit deposit has no order-0 form
    const void* fn = mode == kPushReal    ? reinterpret_cast<const void*>(&k_push<T, kPushReal, O>)
                     : mode == kPushTrial ? reinterpret_cast<const void*>(&k_push<T, kPushTrial, O>)
                     : mode == kPushTrialTape
                         ? reinterpret_cast<const void*>(&k_push<T, kPushTrialTape, O>)
                     : mode == kTrialLater
                         ? reinterpret_cast<const void*>(&k_push<T, kTrialLater, O>)
                     : mode == kExplicitDep
                         ? reinterpret_cast<const void*>(&k_push<T, kExplicitDep, OE>)
                         : reinterpret_cast<const void*>(&k_push<T, kDepositOnly, O>);
    if (lds > 65536)   // opt in above 64 KiB (gfx950 offers 160 KiB per workgroup)
      QSP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    switch (mode) {
      case kPushReal:
        hipLaunchKernelGGL((k_push<T, kPushReal, O>), grid, dim3(kBlock), lds, st, g, L, a, ctr);
        break;
      case kPushTrial:
        hipLaunchKernelGGL((k_push<T, kPushTrial, O>), grid, dim3(kBlock), lds, st, g, L, a, ctr);
        break;
      case kPushTrialTape:
        hipLaunchKernelGGL((k_push<T, kPushTrialTape, O>), grid, dim3(kBlock), lds, st, g, L, a,
                           ctr);
        break;
      case kTrialLater:
        hipLaunchKernelGGL((k_push<T, kTrialLater, O>), grid, dim3(kBlock), lds, st, g, L, a, ctr);
        break;
      case kExplicitDep:
        hipLaunchKernelGGL((k_push<T, kExplicitDep, OE>), grid, dim3(kBlock), lds, st, g, L, a, ctr);
        break;
      default:
        hipLaunchKernelGGL((k_push<T, kDepositOnly, O>), grid, dim3(kBlock), lds, st, g, L, a, ctr);
        break;
    }
  };
  with_order(g.order, run);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_import_state(const Geom& g, const Lattice& L, const Particles<T>& p,
                         const double* x, const double* y, const double* ux, const double* uy,
                         const double* psi, const double* w, const double* hist, int k,
                         double dzeta, hipStream_t st) {
  hipLaunchKernelGGL(k_import_state<T>, grid_1d(L.np), dim3(kBlock), 0, st, g, L, p, x, y, ux,
                     uy, psi, w, hist, k, dzeta);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_export_state(const Geom& g, const Lattice& L, const Particles<T>& p, double* x,
                         double* y, double* ux, double* uy, double* psi, double* w,
                         double* hist, int k, hipStream_t st) {
  hipLaunchKernelGGL(k_export_state<T>, grid_1d(L.np), dim3(kBlock), 0, st, g, L, p, x, y, ux,
                     uy, psi, w, hist, k);
  QSP_LAUNCH_CHECK();
}

#define QSP_INST(T)                                                                         \
  template void launch_init_plasma<T>(const Lattice&, const Particles<T>&, double,          \
                                      hipStream_t);                                         \
  template void launch_push<T>(const Geom&, const Lattice&, const PushArgs<T>&, PushMode,   \
                               DevCounters*, hipStream_t);                                  \
  template void launch_import_state<T>(const Geom&, const Lattice&, const Particles<T>&,    \
                                       const double*, const double*, const double*,         \
                                       const double*, const double*, const double*,         \
                                       const double*, int, double, hipStream_t);            \
  template void launch_export_state<T>(const Geom&, const Lattice&, const Particles<T>&,    \
                                       double*, double*, double*, double*, double*,         \
                                       double*, double*, int, hipStream_t);
QSP_INST(float)
QSP_INST(double)
#undef QSP_INST

}  // namespace qsp
