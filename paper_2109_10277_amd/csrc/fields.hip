// Small grid kernels of the slice loop: buffer clears, the predictor-corrector
// initial guess and bookkeeping, output copies and layout conversions.
#include "common.hpp"
#include "kernels.hpp"
#include "partials.hpp"

namespace qsp {

namespace {

dim3 grid_for(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 65536) b = 65536;
  if (b == 0) b = 1;
  return dim3(static_cast<unsigned>(b));
}

template <typename T>
__global__ void k_zero(T* p, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = T(0);
}

// B^(0) = 2 B_{k-1} - B_{k-2} (linear extrapolation from the two previous
// slices); also opens the predictor-corrector of the slice.
template <typename T>
__global__ void k_guess(size_t n, T* bx, T* by, const T* bx1, const T* by1, const T* bx2,
                        const T* by2, DevCounters* ctr) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctr->pc_done = 0u;
    ctr->pc_iters = 0u;
    ctr->pc_resid = 0.0;
  }
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    bx[i] = T(2) * bx1[i] - bx2[i];
    by[i] = T(2) * by1[i] - by2[i];
  }
}

// explicit beam current of a slice: an ultra-relativistic beam has
// rho_b = Jz_b and rho_b - Jz_b = 0, so the plane is added to Jz (and to a
// separate rho channel if one is kept)
__global__ void k_add_current(size_t n, const double* src, double* jz, double* rho) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const double v = src[i];
    jz[i] += v;
    if (rho) rho[i] += v;
  }
}

__global__ void k_slice_end(DevCounters* ctr, int32_t* iters_out, int32_t* iters_own,
                            double* resid_out, double tol, int max_iter, int budgeted,
                            const double* pc_partial, int pc_nblk) {
  if (pc_partial && !ctr->pc_done) partials::pc_consume(pc_partial, pc_nblk, tol, ctr, true);
  if (threadIdx.x != 0) return;
  const double r = ctr->pc_resid;
  if (iters_out) *iters_out = static_cast<int32_t>(ctr->pc_iters);
  if (iters_own) *iters_own = static_cast<int32_t>(ctr->pc_iters);
  if (resid_out) *resid_out = r;
  if (r > ctr->max_resid || r != r) ctr->max_resid = r;
  if (tol > 0.0 && !ctr->pc_done) {
    if (static_cast<int>(ctr->pc_iters) >= max_iter) ctr->pc_not_converged += 1ull;
    else if (budgeted) ctr->budget_short += 1u;
  }
}

__global__ void k_out_copy(Geom g, OutCopy c) {
  const int id = blockIdx.y;
  const int kind = c.kind[id];
  const int nx = g.nx, ny = g.ny;
  const size_t total = kind == 0 ? static_cast<size_t>(nx + 1) * (ny + 1)
                                 : (kind == 1 ? static_cast<size_t>(nx + 1) : 1);
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<size_t>(gridDim.x) * blockDim.x) {
    int i, j;
    if (kind == 0) {
      i = static_cast<int>(e % (nx + 1));
      j = static_cast<int>(e / (nx + 1));
    } else if (kind == 1) {
      i = static_cast<int>(e);
      j = ny / 2;
    } else {
      i = nx / 2;
      j = ny / 2;
    }
    const bool stored = i < nx && j < ny;
    const bool interior = i > 0 && j > 0 && i < nx && j < ny;
    double v = 0.0;
    if (stored) {
      const size_t o = static_cast<size_t>(j) * nx + i;
      v = c.is_double[id] ? static_cast<const double*>(c.src[id])[o]
                          : static_cast<double>(static_cast<const float*>(c.src[id])[o]);
      if (c.src2[id]) v += c.src2[id][o];
    }
    if (interior) {
      if (c.add_beam[id]) v -= c.beam_amp * c.bgx[i] * c.bgy[j];
      if (c.add_ion[id]) v += c.ionx ? c.n0 * c.ionx[i] * c.iony[j] : c.n0;
    }
    if (c.is_double[id])
      static_cast<double*>(c.dst[id])[e] = v;
    else
      static_cast<float*>(c.dst[id])[e] = static_cast<float>(v);
  }
}

template <typename S, typename T>
__global__ void k_from_nodes(Geom g, const S* src, T* dst) {
  const size_t n = static_cast<size_t>(g.nx) * g.ny;
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int i = static_cast<int>(e % g.nx), j = static_cast<int>(e / g.nx);
    const bool interior = i > 0 && j > 0;
    dst[e] = interior ? static_cast<T>(src[static_cast<size_t>(j) * (g.nx + 1) + i]) : T(0);
  }
}

template <typename T>
__global__ void k_to_nodes(Geom g, const T* src, double* dst) {
  const size_t n = static_cast<size_t>(g.nx + 1) * (g.ny + 1);
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int i = static_cast<int>(e % (g.nx + 1)), j = static_cast<int>(e / (g.nx + 1));
    dst[e] = (i < g.nx && j < g.ny) ? static_cast<double>(src[static_cast<size_t>(j) * g.nx + i])
                                    : 0.0;
  }
}

template <typename T>
__global__ void k_to_nodes_t(Geom g, const T* src, T* dst) {
  const size_t n = static_cast<size_t>(g.nx + 1) * (g.ny + 1);
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int i = static_cast<int>(e % (g.nx + 1)), j = static_cast<int>(e / (g.nx + 1));
    dst[e] = (i < g.nx && j < g.ny) ? src[static_cast<size_t>(j) * g.nx + i] : T(0);
  }
}

}  // namespace

template <typename T>
void launch_to_nodes_t(const Geom& g, const T* src, T* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_to_nodes_t<T>, grid_for(static_cast<size_t>(g.nx + 1) * (g.ny + 1)),
                     dim3(kBlock), 0, st, g, src, dst);
  QSP_LAUNCH_CHECK();
}

void launch_zero_int(int* p, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero<int>, grid_for(n), dim3(kBlock), 0, st, p, n);
  QSP_LAUNCH_CHECK();
}

void launch_zero(double* p, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero<double>, grid_for(n), dim3(kBlock), 0, st, p, n);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_zero_t(T* p, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero<T>, grid_for(n), dim3(kBlock), 0, st, p, n);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_guess(const Geom& g, T* bx, T* by, const T* bx1, const T* by1, const T* bx2,
                  const T* by2, DevCounters* ctr, hipStream_t st) {
  const size_t n = static_cast<size_t>(g.nx) * g.ny;
  hipLaunchKernelGGL(k_guess<T>, grid_for(n), dim3(kBlock), 0, st, n, bx, by, bx1, by1, bx2,
                     by2, ctr);
  QSP_LAUNCH_CHECK();
}

void launch_add_current(size_t n, const double* src, double* jz, double* rho, hipStream_t st) {
  hipLaunchKernelGGL(k_add_current, grid_for(n), dim3(kBlock), 0, st, n, src, jz, rho);
  QSP_LAUNCH_CHECK();
}

void launch_slice_end(DevCounters* ctr, int32_t* iters_out, int32_t* iters_own, double* resid_out,
                      double tol, int max_iter, int budgeted, const double* pc_partial, int pc_nblk,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_slice_end, dim3(1), dim3(kBlock), 0, st, ctr, iters_out, iters_own,
                     resid_out, tol, max_iter, budgeted, pc_partial, pc_nblk);
  QSP_LAUNCH_CHECK();
}

void launch_out_copy(const Geom& g, const OutCopy& c, hipStream_t st) {
  if (c.count == 0) return;
  const size_t plane = static_cast<size_t>(g.nx + 1) * (g.ny + 1);
  size_t b = (plane + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_out_copy, dim3(static_cast<unsigned>(b), c.count), dim3(kBlock), 0, st,
                     g, c);
  QSP_LAUNCH_CHECK();
}

template <typename S, typename T>
void launch_from_nodes(const Geom& g, const S* src, T* dst, hipStream_t st) {
  hipLaunchKernelGGL((k_from_nodes<S, T>), grid_for(static_cast<size_t>(g.nx) * g.ny), dim3(kBlock),
                     0, st, g, src, dst);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_to_nodes(const Geom& g, const T* src, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_to_nodes<T>, grid_for(static_cast<size_t>(g.nx + 1) * (g.ny + 1)),
                     dim3(kBlock), 0, st, g, src, dst);
  QSP_LAUNCH_CHECK();
}

#define QSP_INST(T)                                                                       \
  template void launch_zero_t<T>(T*, size_t, hipStream_t);                                \
  template void launch_guess<T>(const Geom&, T*, T*, const T*, const T*, const T*,        \
                                const T*, DevCounters*, hipStream_t);                     \
  template void launch_from_nodes<double, T>(const Geom&, const double*, T*, hipStream_t); \
  template void launch_to_nodes<T>(const Geom&, const T*, double*, hipStream_t);        \
  template void launch_to_nodes_t<T>(const Geom&, const T*, T*, hipStream_t);
QSP_INST(float)
QSP_INST(double)
#undef QSP_INST
template void launch_from_nodes<float, float>(const Geom&, const float*, float*, hipStream_t);

}  // namespace qsp
