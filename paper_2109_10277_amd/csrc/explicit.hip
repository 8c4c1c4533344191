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
// One iteration m is four launches:
//   matvec(m)  p_m = z_{m-1} + beta p_{m-1}, q_m = A p_m, partial p.q
//   update(m)  alpha_m = rho_{m-1} / (p.q); x += alpha p, r -= alpha q,
//              B = x, partial r.r, forward sine transform along x of -r
//   column     transform along y, division by (lambda - c0), inverse along y
//   rowinv(m)  residual test; inverse transform along x -> z_m = M^-1 r_m,
//              partials of z.r and z.q
// Dot products leave one partial sum per workgroup, which the next kernel
// adds up in every workgroup in the same order: no atomics and no device-
// wide fences inside the solve (a fence per workgroup writes back the XCD's
// L2).  The scalars a later kernel needs are kept by workgroup 0 in
// alternating slots.  After convergence every kernel returns at once.
#include "dst_impl.hpp"
#include "partials.hpp"

namespace qsp {

using namespace dst_detail;

namespace {

__device__ inline bool first_thread() {
  return blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
}

// relative residual of both systems and the stop decision
__device__ inline double rel_residual(double rr, double bn) {
  return bn > 0.0 ? sqrt(rr / bn) : (rr == 0.0 ? 0.0 : INFINITY);
}

__device__ inline bool stops(double rr, double res, double tol) {
  return rr == 0.0 || (tol > 0.0 && res < tol) || !isfinite(res);
}

__device__ inline void record_residual(DevCounters* ctr, double rr, double bn, int iters, bool stop,
                                       double res) {
  ctr->pc_resid = res;
  ctr->pc_iters = static_cast<unsigned int>(iters);
  if (iters > 0) ctr->pc_iterations += 1ull;
  if (!isfinite(res) || !isfinite(rr) || !isfinite(bn)) ctr->nonfinite = 1u;
  if (stop) ctr->pc_done = 1u;
}

}  // namespace

// Set-up: right-hand side b = -R, x0 = the initial guess held in B,
// r0 = b - A x0, partials of ||b||^2 and ||r0||^2, and the forward
// transform along x of -r0.
template <typename T, int LOGN>
__global__ void __launch_bounds__(kBlock, dst_blocks_per_cu(LOGN, sizeof(T)))
k_expl_setup(Geom g, ExplicitArgs<T> a, AxisTables<T> tx, DevCounters* ctr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  const int n = g.nx, ny = g.ny;
  const int R = g.rr;
  const int ppitch = pair_pitch<T>(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables<T, LOGN>(tx, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
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
    buf[RowLay<T, LOGN>::rpos(n, ppitch, rr, i)] = static_cast<T>(-r0);
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  rows_to_plane<T, 0, LOGN>(g, R, j0, buf, ppitch, a.fwd + fld * plane);
  double v[2] = {bn, rn};
  partials::store<2>(v, a.part_s, fld * (ny / R) + blockIdx.x);
}

// Residual test of r_m (partials of the set-up or of update(m)), then the
// inverse transform along x of the column-pass output: z_m = M^-1 r_m, with
// partials of z.r and z.q per system.
template <typename T, int LOGN>
__global__ void __launch_bounds__(kBlock, dst_blocks_per_cu(LOGN, sizeof(T)))
k_expl_rowinv(Geom g, ExplicitArgs<T> a, AxisTables<T> tx, DevCounters* ctr) {
  if (ctr->pc_done) return;
  const int n = g.nx, ny = g.ny;
  const int R = g.rr;
  const int nblk = 2 * (ny / R);
  double bn, rr;
  if (a.it == 0) {
    double t[2];
    partials::sum<2>(a.part_s, nblk, t);
    bn = t[0];
    rr = t[1];
  } else {
    double t[1];
    partials::sum<1>(a.part_u, nblk, t);
    bn = a.s->bnorm2;
    rr = t[0];
  }
  const double res = rel_residual(rr, bn);
  const bool stop = stops(rr, res, a.tol);
  if (first_thread()) {
    if (a.it == 0) a.s->bnorm2 = bn;
    record_residual(ctr, rr, bn, a.it, stop, res);
  }
  if (stop) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  const int ppitch = pair_pitch<T>(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables<T, LOGN>(tx, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int fld = blockIdx.y;
  const int j0 = blockIdx.x * R;
  const size_t plane = static_cast<size_t>(n) * ny;
  const int lx = g.lx;
  plane_to_rows<T, 0, LOGN>(g, R, j0, a.col + fld * plane, buf, ppitch);
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  T* z = a.z + fld * plane;
  const double* r = a.r + fld * plane;
  const double* q = a.q + fld * plane;
  const bool with_q = a.it > 0;
  double zr = 0.0, zq = 0.0;
  for_elems(R * n, [&](int e) {
    const int rw = e >> lx, i = e & (n - 1);
    const int j = j0 + rw;
    const int o = j * n + i;
    const T u = buf[RowLay<T, LOGN>::rpos(n, ppitch, rw, i)];
    const T zv = (i > 0 && j > 0) ? u : T(0);
    z[o] = zv;
    zr += static_cast<double>(zv) * r[o];
    if (with_q) zq += static_cast<double>(zv) * q[o];
  });
  double v[4] = {fld == 0 ? zr : 0.0, fld == 1 ? zr : 0.0, fld == 0 ? zq : 0.0,
                 fld == 1 ? zq : 0.0};
  partials::store<4>(v, a.part_z, fld * (ny / R) + blockIdx.x);
}

// matvec(it): rho_{it-1} = z.r and the Polak-Ribiere
// beta = -alpha_{it-1} (z.q) / rho_{it-2}; p = z + beta p_old (p_old unused
// in the first iteration), q = A p and partials of p.q.  Grid (ny/R, 2).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_expl_matvec(Geom g, ExplicitArgs<T> a, DevCounters* ctr) {
  if (ctr->pc_done) return;
  const int n = g.nx, ny = g.ny;
  const int R = g.rr;
  const int nblk = 2 * (ny / R);
  const int fld = blockIdx.y;
  double t[4];
  partials::sum<4>(a.part_z, nblk, t);
  const int it = a.it;
  const bool use_old = it > 1;
  double beta = 0.0;
  if (use_old) {
    const double rho_prev = a.s->rho[it & 1][fld];          // rho_{it-2}
    const double alpha = a.s->alpha[(it - 1) & 1][fld];     // alpha_{it-1}
    beta = rho_prev != 0.0 ? -alpha * t[2 + fld] / rho_prev : 0.0;
  }
  if (first_thread()) {
    a.s->rho[(it - 1) & 1][0] = t[0];                      // rho_{it-1}
    a.s->rho[(it - 1) & 1][1] = t[1];
  }
  const size_t plane = static_cast<size_t>(n) * ny;
  const T* z = a.z + fld * plane;
  const double* pold = a.p[(it + 1) & 1] + fld * plane;
  double* pnew = a.p[it & 1] + fld * plane;
  double* q = a.q + fld * plane;
  const double* chi = a.chi;
  const double ihx2 = 1.0 / (g.hx * g.hx), ihy2 = 1.0 / (g.hy * g.hy);
  const int j0 = blockIdx.x * R;
  const int lx = g.lx;
  double pq = 0.0;
  for_elems(R * n, [&](int e) {
    const int rw = e >> lx, i = e & (n - 1);
    const int j = j0 + rw;
    const int o = j * n + i;
    // neighbours with clamped indices; nodes on or beyond the Dirichlet
    // boundary are zero
    const int ow = i > 0 ? o - 1 : o, oe = i + 1 < n ? o + 1 : o;
    const int os = j > 0 ? o - n : o, on = j + 1 < ny ? o + n : o;
    double pc = static_cast<double>(z[o]), pw = static_cast<double>(z[ow]);
    double pe = static_cast<double>(z[oe]), ps = static_cast<double>(z[os]);
    double pn = static_cast<double>(z[on]);
    if (use_old) {
      pc += beta * pold[o];
      pw += beta * pold[ow];
      pe += beta * pold[oe];
      ps += beta * pold[os];
      pn += beta * pold[on];
    }
    const bool inner = i > 0 && j > 0;
    pc = inner ? pc : 0.0;
    pw = i > 1 ? pw : 0.0;
    pe = i + 1 < n ? pe : 0.0;
    ps = j > 1 ? ps : 0.0;
    pn = j + 1 < ny ? pn : 0.0;
    const double lap = (pe - 2.0 * pc + pw) * ihx2 + (pn - 2.0 * pc + ps) * ihy2;
    const double qv = inner ? -lap + chi[o] * pc : 0.0;
    pnew[o] = pc;
    q[o] = qv;
    pq += pc * qv;
  });
  double v[2] = {fld == 0 ? pq : 0.0, fld == 1 ? pq : 0.0};
  partials::store<2>(v, a.part_m, fld * (ny / R) + blockIdx.x);
}

// update(it): alpha = rho_{it-1} / (p.q); x += alpha p, r -= alpha q, B = x;
// partials of r.r; forward transform along x of -r for the preconditioner.
template <typename T, int LOGN>
__global__ void __launch_bounds__(kBlock, dst_blocks_per_cu(LOGN, sizeof(T)))
k_expl_update(Geom g, ExplicitArgs<T> a, AxisTables<T> tx, DevCounters* ctr) {
  if (ctr->pc_done) return;
  const int n = g.nx, ny = g.ny;
  const int R = g.rr;
  const int nblk = 2 * (ny / R);
  const int fld = blockIdx.y;
  const int it = a.it;
  double t[2];
  partials::sum<2>(a.part_m, nblk, t);
  const double rho = a.s->rho[(it - 1) & 1][fld];
  const double alpha = t[fld] > 0.0 ? rho / t[fld] : 0.0;
  if (first_thread()) {
    a.s->alpha[it & 1][0] = t[0] > 0.0 ? a.s->rho[(it - 1) & 1][0] / t[0] : 0.0;
    a.s->alpha[it & 1][1] = t[1] > 0.0 ? a.s->rho[(it - 1) & 1][1] / t[1] : 0.0;
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  const int ppitch = pair_pitch<T>(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables<T, LOGN>(tx, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int j0 = blockIdx.x * R;
  const size_t plane = static_cast<size_t>(n) * ny;
  const double* p = a.p[it & 1] + fld * plane;
  const double* q = a.q + fld * plane;
  double* x = a.x + fld * plane;
  double* r = a.r + fld * plane;
  T* B = a.b[fld];
  const int lx = g.lx;
  double rn = 0.0;
  for_elems(R * n, [&](int e) {
    const int rw = e >> lx, i = e & (n - 1);
    const int j = j0 + rw;
    const int o = j * n + i;
    const bool inner = i > 0 && j > 0;
    const double xv = inner ? x[o] + alpha * p[o] : 0.0;
    const double rv = inner ? r[o] - alpha * q[o] : 0.0;
    x[o] = xv;
    r[o] = rv;
    B[o] = static_cast<T>(xv);
    rn += rv * rv;
    buf[RowLay<T, LOGN>::rpos(n, ppitch, rw, i)] = static_cast<T>(-rv);
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  rows_to_plane<T, 0, LOGN>(g, R, j0, buf, ppitch, a.fwd + fld * plane);
  double v[1] = {rn};
  partials::store<1>(v, a.part_u, fld * (ny / R) + blockIdx.x);
}

// Residual test after the last iteration (one workgroup).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_expl_close(Geom g, ExplicitArgs<T> a, DevCounters* ctr) {
  if (ctr->pc_done) return;
  double t[1];
  partials::sum<1>(a.part_u, 2 * (g.ny / g.rr), t);
  const double bn = a.s->bnorm2;
  const double res = rel_residual(t[0], bn);
  if (threadIdx.x == 0) record_residual(ctr, t[0], bn, a.it, stops(t[0], res, a.tol), res);
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
  return static_cast<size_t>(g.rr / 2) * pair_pitch<T>(g.nx) * sizeof(T) + table_bytes<T>(g.nx);
}

}  // namespace

// partial records of one row-blocked grid: one per workgroup of (ny/rr, 2)
int explicit_partial_count(const Geom& g) { return 2 * (g.ny / g.rr); }

template <typename T>
void launch_explicit(const Geom& g, const ExplicitArgs<T>& a, ExplicitStep step,
                     const AxisTables<T>& tx, DevCounters* ctr, hipStream_t st) {
  const int R = g.rr;
  const size_t lds = row_lds<T>(g);
  if (step == kExplMatvec) {
    hipLaunchKernelGGL((k_expl_matvec<T>), dim3(g.ny / R, 2), dim3(kBlock), 0, st, g, a, ctr);
    QSP_LAUNCH_CHECK();
    return;
  }
  if (step == kExplClose) {
    hipLaunchKernelGGL((k_expl_close<T>), dim3(1), dim3(kBlock), 0, st, g, a, ctr);
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
