// Explicit Bx/By field solver (HiPACE++, arXiv:2109.10277 Sec. III.B, the
// second option of the Bx/By solver): with d_zeta J_perp integrated along
// the particle orbits, eq. (bxby) becomes
//   (lap - chi) Bx = -d_y Jz + DJy,   (lap - chi) By = d_x Jz - DJx,
// a Helmholtz-like equation whose coefficient chi varies from node to node.
// It is solved on the grid, without further particle passes, by conjugate
// gradients on A = -lap + chi (symmetric positive definite for chi >= 0)
// preconditioned by the constant-coefficient operator M = -lap + c0, which
// the sine transform inverts exactly.  Both components run as one batch of
// two systems.  Krylov vectors are FP64; the preconditioner runs in the
// field precision T, so the Polak-Ribiere form of beta is used (it tolerates
// an inexact preconditioner).
//
// One iteration is four launches:
//   matvec    p = z + beta p_old, q = A p, alpha = rho / (p.q)
//   update    x += alpha p, r -= alpha q, B = x, residual, then the forward
//             sine transform along x of -r
//   column    transform along y, division by (lambda - c0), inverse along y
//   rowinv    inverse transform along x -> z = M^-1 r; rho = z.r and
//             beta = -alpha (z.q) / rho_old
// Every kernel returns at once after convergence (device-side flag).
#include "dst_impl.hpp"

namespace qsp {

using namespace dst_detail;

namespace {

// Adds v[0..NV-1] over the workgroup and stores the sums at partial[bid*NV];
// the last of nblk workgroups to arrive returns true with the totals over
// all workgroups in tot (valid in thread 0), summed in a fixed order.
template <int NV>
__device__ bool reduce_last(double (&v)[NV], double* partial, int bid, int nblk,
                            unsigned int* arrived, double (&tot)[NV]) {
  __shared__ double red[NV][kBlock / 64];
  __shared__ bool last;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wave] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) s += red[k][w];
      partial[static_cast<size_t>(bid) * NV + k] = s;
    }
    __threadfence();
    const unsigned int prev = atomicAdd(arrived, 1u);
    last = (prev == static_cast<unsigned int>(nblk - 1));
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double t[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) t[k] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kBlock)
#pragma unroll
    for (int k = 0; k < NV; ++k) t[k] += partial[static_cast<size_t>(b) * NV + k];
#pragma unroll
  for (int k = 0; k < NV; ++k)
    for (int off = 32; off > 0; off >>= 1) t[k] += __shfl_down(t[k], off, 64);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wave] = t[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) s += red[k][w];
      tot[k] = s;
    }
    *arrived = 0u;
  }
  return true;
}

// relative residual ||r|| / ||b|| of both systems together
__device__ inline void close_residual(DevCounters* ctr, double rn, double bn, double tol) {
  const double res = bn > 0.0 ? sqrt(rn / bn) : (rn == 0.0 ? 0.0 : INFINITY);
  if (!isfinite(res) || !isfinite(rn) || !isfinite(bn)) ctr->nonfinite = 1u;
  ctr->pc_resid = res;
  if (rn == 0.0 || (tol > 0.0 && res < tol)) ctr->pc_done = 1u;
}

}  // namespace

// Set-up: right-hand side b = -R, x0 = the initial guess held in B,
// r0 = b - A x0, ||b||^2, and the forward transform along x of -r0.
template <typename T, int LOGN>
__global__ void __launch_bounds__(kBlock, dst_blocks_per_cu(LOGN, sizeof(T)))
k_expl_setup(Geom g, ExplicitArgs<T> a, AxisTables<T> tx, DevCounters* ctr) {
  extern __shared__ unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  const int n = g.nx, ny = g.ny;
  const int R = g.rr;
  const int ppitch = Pad<T>::pitch(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables(tx, n, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int fld = blockIdx.y;
  const int j0 = blockIdx.x * R;
  const size_t plane = static_cast<size_t>(n) * ny;
  const double ihx = 0.5 / g.hx, ihy = 0.5 / g.hy;
  const double ihx2 = 1.0 / (g.hx * g.hx), ihy2 = 1.0 / (g.hy * g.hy);
  const double amp = a.beam_amp;
  const T* B = a.b[fld];
  double* x = a.x + fld * plane;
  double* r = a.r + fld * plane;
  const int lx = g.lx;
  double bn = 0.0, rn = 0.0;
  for_elems(R * n, [&](int e) {
    const int rr = e >> lx, i = e & (n - 1);
    const int j = j0 + rr;
    const int o = j * n + i;
    const bool inner = i > 0 && j > 0;
    double rhs;
    if (fld == 0) {
      // R_x = -d_y Jz + DJy (the Gaussian beam's Jz = -amp gx gy on the fly)
      const int js = j > 0 ? j - 1 : 0;
      const double zs = a.jz[js * n + i], zn = a.jz[(j + 1 < ny ? j + 1 : j) * n + i];
      const double gx = a.bgx[i], gs = a.bgy[js], gn = a.bgy[j + 1];
      const double jz_s = zs - amp * gx * gs;
      const double jz_n = j + 1 < ny ? zn - amp * gx * gn : 0.0;
      rhs = -(jz_n - jz_s) * ihy + a.djy[o];
    } else {
      // R_y = d_x Jz - DJx
      const int iw = i > 0 ? i - 1 : 0;
      const double zw = a.jz[j * n + iw], ze = a.jz[j * n + (i + 1 < n ? i + 1 : i)];
      const double gy = a.bgy[j], gw = a.bgx[iw], ge = a.bgx[i + 1];
      const double jz_w = zw - amp * gw * gy;
      const double jz_e = i + 1 < n ? ze - amp * ge * gy : 0.0;
      rhs = (jz_e - jz_w) * ihx - a.djx[o];
    }
    // A x0 with x0 = 0 on and beyond the Dirichlet nodes
    const double x0 = static_cast<double>(B[o]);
    const double xe = i + 1 < n ? static_cast<double>(B[i + 1 < n ? o + 1 : o]) : 0.0;
    const double xw = i > 1 ? static_cast<double>(B[i > 0 ? o - 1 : o]) : 0.0;
    const double xn = j + 1 < ny ? static_cast<double>(B[j + 1 < ny ? o + n : o]) : 0.0;
    const double xs = j > 1 ? static_cast<double>(B[j > 0 ? o - n : o]) : 0.0;
    const double ax0 = -((xe - 2.0 * x0 + xw) * ihx2 + (xn - 2.0 * x0 + xs) * ihy2) + a.chi[o] * x0;
    const double b = inner ? -rhs : 0.0;
    const double r0 = inner ? b - ax0 : 0.0;
    x[o] = inner ? x0 : 0.0;
    r[o] = r0;
    bn += b * b;
    rn += r0 * r0;
    buf[Pad<T>::rpos(n, ppitch, rr, i)] = static_cast<T>(-r0);
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  T* out = a.fwd + fld * plane;
  for_elems(R * n, [&](int e) {
    const int rr = e >> lx, i = e & (n - 1);
    out[(j0 + rr) * n + i] = buf[Pad<T>::rpos(n, ppitch, rr, i)];
  });
  double v[2] = {bn, rn}, tot[2];
  const int nrb = ny / R;
  if (reduce_last<2>(v, a.partial, fld * nrb + blockIdx.x, 2 * nrb, &a.s->blocks_arrived, tot) &&
      threadIdx.x == 0) {
    a.s->bnorm2 = tot[0];
    close_residual(ctr, tot[1], tot[0], a.tol);
  }
}

// Inverse transform along x of the column-pass output: z = M^-1 r; then
// rho = z.r and, from the second round on, the Polak-Ribiere beta.
template <typename T, int LOGN>
__global__ void __launch_bounds__(kBlock, dst_blocks_per_cu(LOGN, sizeof(T)))
k_expl_rowinv(Geom g, ExplicitArgs<T> a, AxisTables<T> tx, DevCounters* ctr) {
  if (ctr->pc_done) return;
  extern __shared__ unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  const int n = g.nx, ny = g.ny;
  const int R = g.rr;
  const int ppitch = Pad<T>::pitch(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables(tx, n, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int fld = blockIdx.y;
  const int j0 = blockIdx.x * R;
  const size_t plane = static_cast<size_t>(n) * ny;
  const T* in = a.col + fld * plane;
  const int lx = g.lx;
  for_elems(R * n, [&](int e) {
    const int rr = e >> lx, i = e & (n - 1);
    buf[Pad<T>::rpos(n, ppitch, rr, i)] = in[(j0 + rr) * n + i];
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  T* z = a.z + fld * plane;
  const double* r = a.r + fld * plane;
  const double* q = a.q + fld * plane;
  const bool with_q = a.it > 0;
  double zr = 0.0, zq = 0.0;
  for_elems(R * n, [&](int e) {
    const int rr = e >> lx, i = e & (n - 1);
    const int j = j0 + rr;
    const int o = j * n + i;
    const T u = buf[Pad<T>::rpos(n, ppitch, rr, i)];
    const T zv = (i > 0 && j > 0) ? u : T(0);
    z[o] = zv;
    zr += static_cast<double>(zv) * r[o];
    if (with_q) zq += static_cast<double>(zv) * q[o];
  });
  double v[4] = {fld == 0 ? zr : 0.0, fld == 1 ? zr : 0.0, fld == 0 ? zq : 0.0,
                 fld == 1 ? zq : 0.0};
  double tot[4];
  const int nrb = ny / R;
  if (reduce_last<4>(v, a.partial, fld * nrb + blockIdx.x, 2 * nrb, &a.s->blocks_arrived, tot) &&
      threadIdx.x == 0) {
    for (int s = 0; s < 2; ++s) {
      const double rho_old = a.s->rho[s];
      a.s->beta[s] = (with_q && rho_old != 0.0) ? -a.s->alpha[s] * tot[2 + s] / rho_old : 0.0;
      a.s->rho[s] = tot[s];
    }
  }
}

// p = z + beta p_old (p_old unused in the first iteration), q = A p and
// alpha = rho / (p.q) per system.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_expl_matvec(Geom g, ExplicitArgs<T> a, DevCounters* ctr) {
  if (ctr->pc_done) return;
  const int n = g.nx, ny = g.ny;
  const size_t plane = static_cast<size_t>(n) * ny;
  const int fld = blockIdx.y;
  const T* z = a.z + fld * plane;
  const double* pold = a.p[(a.it + 1) & 1] + fld * plane;
  double* pnew = a.p[a.it & 1] + fld * plane;
  double* q = a.q + fld * plane;
  const double beta = a.it > 1 ? a.s->beta[fld] : 0.0;
  const bool use_old = a.it > 1;
  const double ihx2 = 1.0 / (g.hx * g.hx), ihy2 = 1.0 / (g.hy * g.hy);
  auto P = [&](int i, int j) -> double {
    if (i < 1 || i >= n || j < 1 || j >= ny) return 0.0;
    const size_t o = static_cast<size_t>(j) * n + i;
    return static_cast<double>(z[o]) + (use_old ? beta * pold[o] : 0.0);
  };
  double pq = 0.0;
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < plane;
       e += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int i = static_cast<int>(e % n), j = static_cast<int>(e / n);
    const double pc = P(i, j);
    const double lap = (P(i + 1, j) - 2.0 * pc + P(i - 1, j)) * ihx2 +
                       (P(i, j + 1) - 2.0 * pc + P(i, j - 1)) * ihy2;
    const bool inner = i > 0 && j > 0;
    const double qv = inner ? -lap + a.chi[e] * pc : 0.0;
    pnew[e] = pc;
    q[e] = qv;
    pq += pc * qv;
  }
  double v[2] = {fld == 0 ? pq : 0.0, fld == 1 ? pq : 0.0}, tot[2];
  if (reduce_last<2>(v, a.partial, fld * gridDim.x + blockIdx.x, 2 * gridDim.x,
                     &a.s->blocks_arrived, tot) &&
      threadIdx.x == 0) {
    for (int s = 0; s < 2; ++s) a.s->alpha[s] = tot[s] > 0.0 ? a.s->rho[s] / tot[s] : 0.0;
  }
}

// x += alpha p, r -= alpha q, B = x; residual; forward transform along x
// of -r for the preconditioner.
template <typename T, int LOGN>
__global__ void __launch_bounds__(kBlock, dst_blocks_per_cu(LOGN, sizeof(T)))
k_expl_update(Geom g, ExplicitArgs<T> a, AxisTables<T> tx, DevCounters* ctr) {
  if (ctr->pc_done) return;
  extern __shared__ unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  const int n = g.nx, ny = g.ny;
  const int R = g.rr;
  const int ppitch = Pad<T>::pitch(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables(tx, n, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int fld = blockIdx.y;
  const int j0 = blockIdx.x * R;
  const size_t plane = static_cast<size_t>(n) * ny;
  const double alpha = a.s->alpha[fld];
  const double* p = a.p[a.it & 1] + fld * plane;
  const double* q = a.q + fld * plane;
  double* x = a.x + fld * plane;
  double* r = a.r + fld * plane;
  T* B = a.b[fld];
  const int lx = g.lx;
  double rn = 0.0;
  for_elems(R * n, [&](int e) {
    const int rr = e >> lx, i = e & (n - 1);
    const int j = j0 + rr;
    const int o = j * n + i;
    const bool inner = i > 0 && j > 0;
    const double xv = inner ? x[o] + alpha * p[o] : 0.0;
    const double rv = inner ? r[o] - alpha * q[o] : 0.0;
    x[o] = xv;
    r[o] = rv;
    B[o] = static_cast<T>(xv);
    rn += rv * rv;
    buf[Pad<T>::rpos(n, ppitch, rr, i)] = static_cast<T>(-rv);
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  T* out = a.fwd + fld * plane;
  for_elems(R * n, [&](int e) {
    const int rr = e >> lx, i = e & (n - 1);
    out[(j0 + rr) * n + i] = buf[Pad<T>::rpos(n, ppitch, rr, i)];
  });
  double v[1] = {rn}, tot[1];
  const int nrb = ny / R;
  if (reduce_last<1>(v, a.partial, fld * nrb + blockIdx.x, 2 * nrb, &a.s->blocks_arrived, tot) &&
      threadIdx.x == 0) {
    ctr->pc_iters += 1u;
    ctr->pc_iterations += 1ull;
    close_residual(ctr, tot[0], a.s->bnorm2, a.tol);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

void allow_lds_e(const void* fn, size_t lds) {
  if (lds > 65536)
    QSP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(lds)));
}

template <typename T>
size_t row_lds(const Geom& g) {
  return static_cast<size_t>(g.rr / 2) * Pad<T>::pitch(g.nx) * sizeof(T) + table_bytes<T>(g.nx);
}

}  // namespace

int explicit_matvec_blocks(const Geom& g) {
  const size_t plane = static_cast<size_t>(g.nx) * g.ny;
  size_t b = (plane + kBlock - 1) / kBlock;
  if (b > 512) b = 512;
  return static_cast<int>(b);
}

int explicit_partial_count(const Geom& g) {
  const int rows = 2 * (g.ny / g.rr) * 4;
  const int mv = 2 * explicit_matvec_blocks(g) * 2;
  return rows > mv ? rows : mv;
}

template <typename T>
void launch_explicit(const Geom& g, const ExplicitArgs<T>& a, ExplicitStep step,
                     const AxisTables<T>& tx, DevCounters* ctr, hipStream_t st) {
  const int R = g.rr;
  const size_t lds = row_lds<T>(g);
  if (step == kExplMatvec) {
    hipLaunchKernelGGL((k_expl_matvec<T>), dim3(explicit_matvec_blocks(g), 2), dim3(kBlock), 0,
                       st, g, a, ctr);
    QSP_LAUNCH_CHECK();
    return;
  }
  with_logn(g.nx, [&](auto e) {
    constexpr int E = decltype(e)::value;
    switch (step) {
      case kExplSetup:
        allow_lds_e(reinterpret_cast<const void*>(&k_expl_setup<T, E>), lds);
        hipLaunchKernelGGL((k_expl_setup<T, E>), dim3(g.ny / R, 2), dim3(kBlock), lds, st, g, a,
                           tx, ctr);
        break;
      case kExplUpdate:
        allow_lds_e(reinterpret_cast<const void*>(&k_expl_update<T, E>), lds);
        hipLaunchKernelGGL((k_expl_update<T, E>), dim3(g.ny / R, 2), dim3(kBlock), lds, st, g, a,
                           tx, ctr);
        break;
      default:
        allow_lds_e(reinterpret_cast<const void*>(&k_expl_rowinv<T, E>), lds);
        hipLaunchKernelGGL((k_expl_rowinv<T, E>), dim3(g.ny / R, 2), dim3(kBlock), lds, st, g, a,
                           tx, ctr);
        break;
    }
  });
  QSP_LAUNCH_CHECK();
}

template void launch_explicit<float>(const Geom&, const ExplicitArgs<float>&, ExplicitStep,
                                     const AxisTables<float>&, DevCounters*, hipStream_t);
template void launch_explicit<double>(const Geom&, const ExplicitArgs<double>&, ExplicitStep,
                                      const AxisTables<double>&, DevCounters*, hipStream_t);

}  // namespace qsp
