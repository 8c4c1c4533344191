// Macro-particle beams (HiPACE++, arXiv:2109.10277, Sec. III.A): the beam is
// sorted by slice once per box, and inside the slice loop the particles of
// slice k deposit their charge and longitudinal current (zeroth order in
// zeta, CIC transversely) before the field solves, then take one time step
// (second-order drift-kick-drift with a Boris kick) in the fields of slice k
// once those are final.  The slice sort is rocPRIM's stable radix sort.
#include "common.hpp"
#include "kernels.hpp"

#include <rocprim/device/device_radix_sort.hpp>

namespace qsp {

namespace {

dim3 grid_of(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 65535 * 16) b = 65535 * 16;
  return dim3(static_cast<unsigned>(b));
}

__global__ void k_beam_keys(const float* __restrict__ soa, int64_t n, double zeta_hi,
                            double dzeta, int nzeta, int* keys, int* idx) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double z = soa[2 * n + i];
    const double s = rint((zeta_hi - z) / dzeta);   // nearest slice
    int key = nzeta;
    if (s >= 0.0 && s < static_cast<double>(nzeta)) key = static_cast<int>(s);
    keys[i] = key;
    idx[i] = static_cast<int>(i);
  }
}

__global__ void k_beam_count(const int* __restrict__ keys, int64_t n, int* counts) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    atomicAdd(&counts[keys[i]], 1);
}

__global__ void k_beam_permute(const float* __restrict__ in, int64_t n,
                               const int* __restrict__ perm, float* out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t src = perm[i];
#pragma unroll
    for (int c = 0; c < 7; ++c) out[c * n + i] = in[c * n + src];
  }
}

// CIC cell and offset of an absolute position; false outside [lo, lo + n h]
__device__ inline bool cic(double x, double lo, double h, int n, int& i, double& f) {
  const double s = (x - lo) / h;
  if (!(s >= 0.0 && s <= static_cast<double>(n))) return false;
  double fl = floor(s);
  i = static_cast<int>(fl);
  f = s - fl;
  if (i >= n) {
    i = n - 1;
    f = 1.0;
  }
  return true;
}

__device__ inline void add_node(double* p, int i, int j, int nx, int ny, double v) {
  if (i >= 1 && i < nx && j >= 1 && j < ny) unsafeAtomicAdd(p + static_cast<size_t>(j) * nx + i, v);
}

template <typename T>
__device__ inline double node_val(const T* F, int i, int j, int nx, int ny) {
  return (i < nx && j < ny) ? static_cast<double>(F[static_cast<size_t>(j) * nx + i]) : 0.0;
}

template <typename T>
__device__ inline double gather_d(const T* F, int i, int j, double fx, double fy, int nx, int ny) {
  return (1 - fx) * (1 - fy) * node_val(F, i, j, nx, ny) + fx * (1 - fy) * node_val(F, i + 1, j, nx, ny) +
         (1 - fx) * fy * node_val(F, i, j + 1, nx, ny) + fx * fy * node_val(F, i + 1, j + 1, nx, ny);
}

}  // namespace

// rho = q w / (hx hy dzeta), Jz = rho u_z / gamma, rho - Jz written as
// rho (1 + u_perp^2) / (gamma (gamma + u_z)) so that it does not cancel
__global__ void k_beam_deposit(Geom g, const float* __restrict__ soa, int64_t n, int64_t start,
                               int64_t count, double dzeta, double* rho_mjz, double* jz,
                               double* rho) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (t >= count) return;
  const int64_t p = start + t;
  const double x = soa[p], y = soa[n + p];
  const double ux = soa[3 * n + p], uy = soa[4 * n + p], uz = soa[5 * n + p], w = soa[6 * n + p];
  int i, j;
  double fx, fy;
  if (!cic(x, g.x_lo, g.hx, g.nx, i, fx) || !cic(y, g.y_lo, g.hy, g.ny, j, fy)) return;
  const double gam = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
  const double r = -w / (g.hx * g.hy * dzeta);
  const double v[3] = {r * (1.0 + ux * ux + uy * uy) / (gam * (gam + uz)), r * uz / gam, r};
  double* ch[3] = {rho_mjz, jz, rho};
  const double s[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
  const int di[4] = {0, 1, 0, 1}, dj[4] = {0, 0, 1, 1};
  for (int c = 0; c < 3; ++c) {
    if (!ch[c]) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) add_node(ch[c], i + di[q], j + dj[q], g.nx, g.ny, v[c] * s[q]);
  }
}

// one time step of the particles of a slice in that slice's fields
template <typename T>
__global__ void k_beam_push(Geom g, float* soa, int64_t n, int64_t start, int64_t count,
                            SliceFields<T> f, double dt) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (t >= count) return;
  const int64_t p = start + t;
  double u[3] = {soa[3 * n + p], soa[4 * n + p], soa[5 * n + p]};
  const double g0 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const double xh = soa[p] + 0.5 * dt * u[0] / g0;
  const double yh = soa[n + p] + 0.5 * dt * u[1] / g0;
  const double zh = soa[2 * n + p] + 0.5 * dt * (u[2] / g0 - 1.0);
  double E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
  int i, j;
  double fx, fy;
  if (cic(xh, g.x_lo, g.hx, g.nx, i, fx) && cic(yh, g.y_lo, g.hy, g.ny, j, fy)) {
    const double e1 = gather_d(f.exmby, i, j, fx, fy, g.nx, g.ny);
    const double e2 = gather_d(f.eypbx, i, j, fx, fy, g.nx, g.ny);
    B[0] = gather_d(f.bx, i, j, fx, fy, g.nx, g.ny);
    B[1] = gather_d(f.by, i, j, fx, fy, g.nx, g.ny);
    B[2] = gather_d(f.bz, i, j, fx, fy, g.nx, g.ny);
    E[0] = e1 + B[1];
    E[1] = e2 - B[0];
    E[2] = gather_d(f.ez, i, j, fx, fy, g.nx, g.ny);
  }
  const double h = -0.5 * dt;   // q dt / 2 with q = -1
  double um[3], tv[3], sv[3], up[3], un[3];
  for (int c = 0; c < 3; ++c) um[c] = u[c] + h * E[c];
  const double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  for (int c = 0; c < 3; ++c) tv[c] = h * B[c] / gm;
  const double tt = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
  for (int c = 0; c < 3; ++c) sv[c] = 2.0 * tv[c] / (1.0 + tt);
  up[0] = um[0] + (um[1] * tv[2] - um[2] * tv[1]);
  up[1] = um[1] + (um[2] * tv[0] - um[0] * tv[2]);
  up[2] = um[2] + (um[0] * tv[1] - um[1] * tv[0]);
  un[0] = um[0] + (up[1] * sv[2] - up[2] * sv[1]) + h * E[0];
  un[1] = um[1] + (up[2] * sv[0] - up[0] * sv[2]) + h * E[1];
  un[2] = um[2] + (up[0] * sv[1] - up[1] * sv[0]) + h * E[2];
  const double g1 = sqrt(1.0 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
  soa[p] = static_cast<float>(xh + 0.5 * dt * un[0] / g1);
  soa[n + p] = static_cast<float>(yh + 0.5 * dt * un[1] / g1);
  soa[2 * n + p] = static_cast<float>(zh + 0.5 * dt * (un[2] / g1 - 1.0));
  soa[3 * n + p] = static_cast<float>(un[0]);
  soa[4 * n + p] = static_cast<float>(un[1]);
  soa[5 * n + p] = static_cast<float>(un[2]);
}

// ------------------------------------------------------------------ host side
void beam_sort(const float* in, float* out, int64_t n, double zeta_hi, double dzeta, int nzeta,
               BeamScratch& s, std::vector<int64_t>& offsets, hipStream_t st) {
  hipLaunchKernelGGL(k_beam_keys, grid_of(n), dim3(kBlock), 0, st, in, n, zeta_hi, dzeta, nzeta,
                     s.keys_in, s.idx_in);
  QSP_LAUNCH_CHECK();
  int bits = 1;
  while ((1 << bits) <= nzeta) ++bits;
  size_t need = 0;
  QSP_HIP(rocprim::radix_sort_pairs(nullptr, need, s.keys_in, s.keys_out, s.idx_in, s.idx_out,
                                    static_cast<size_t>(n), 0u, static_cast<unsigned>(bits), st));
  if (need > s.temp_bytes) throw std::runtime_error("beam sort scratch too small");
  QSP_HIP(rocprim::radix_sort_pairs(s.temp, need, s.keys_in, s.keys_out, s.idx_in, s.idx_out,
                                    static_cast<size_t>(n), 0u, static_cast<unsigned>(bits), st));
  hipLaunchKernelGGL(k_beam_permute, grid_of(n), dim3(kBlock), 0, st, in, n, s.idx_out, out);
  QSP_LAUNCH_CHECK();
  launch_zero_int(s.counts, nzeta + 1, st);
  hipLaunchKernelGGL(k_beam_count, grid_of(n), dim3(kBlock), 0, st, s.keys_out, n, s.counts);
  QSP_LAUNCH_CHECK();
  std::vector<int> c(nzeta + 1);
  QSP_HIP(hipMemcpyAsync(c.data(), s.counts, (nzeta + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
  QSP_HIP(hipStreamSynchronize(st));
  offsets.assign(nzeta + 2, 0);
  for (int k = 0; k <= nzeta; ++k) offsets[k + 1] = offsets[k] + c[k];
}

size_t beam_sort_temp_bytes(int64_t n, int nzeta) {
  int bits = 1;
  while ((1 << bits) <= nzeta) ++bits;
  size_t need = 0;
  QSP_HIP(rocprim::radix_sort_pairs(nullptr, need, static_cast<int*>(nullptr),
                                    static_cast<int*>(nullptr), static_cast<int*>(nullptr),
                                    static_cast<int*>(nullptr), static_cast<size_t>(n), 0u,
                                    static_cast<unsigned>(bits)));
  return need;
}

void launch_beam_deposit(const Geom& g, const float* soa, int64_t n, int64_t start, int64_t count,
                         double dzeta, double* rho_mjz, double* jz, double* rho, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_beam_deposit, grid_of(count), dim3(kBlock), 0, st, g, soa, n, start, count,
                     dzeta, rho_mjz, jz, rho);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_beam_push(const Geom& g, float* soa, int64_t n, int64_t start, int64_t count,
                      const SliceFields<T>& f, double dt, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_beam_push<T>, grid_of(count), dim3(kBlock), 0, st, g, soa, n, start, count,
                     f, dt);
  QSP_LAUNCH_CHECK();
}

template void launch_beam_push<float>(const Geom&, float*, int64_t, int64_t, int64_t,
                                      const SliceFields<float>&, double, hipStream_t);
template void launch_beam_push<double>(const Geom&, float*, int64_t, int64_t, int64_t,
                                       const SliceFields<double>&, double, hipStream_t);

}  // namespace qsp
