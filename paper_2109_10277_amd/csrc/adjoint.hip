// Adjoint (reverse-mode) kernels of the slice loop.  Every kernel is the
// transpose of a forward step of the HiPACE++ slice routine (arXiv:2109.10277
// Sec. II, III.B) as the forward kernels discretise it:
//   * field gather (shape S of order 1-3)
//                                   -> FP64 scatter of the gathered adjoints
//                                      plus grad-S position terms;
//   * deposit (shape S)             -> gather of the adjoint planes with S and
//                                      grad S;
//   * pusher right-hand side        -> its Jacobian, transposed;
//   * Adams-Bashforth step          -> adjoint history ring (slot s holds the
//                                      adjoint of the f stored in slot s);
//   * (lap - s)^-1, centred d/dx    -> the same solves, D^T = -D.
// Positions are the displacements xi (cell units) of the forward kernels, so
// the position adjoints are per cell.  Particles the step absorbs, dead
// particles and floored 1+Psi are locally constant.
#include "common.hpp"
#include "kernels.hpp"
#include "push_tile.hpp"
#include "shape.hpp"

namespace qsp {

namespace {

__device__ inline void gadd(double* p, double v) { unsafeAtomicAdd(p, v); }

// node value with the Dirichlet nodes (index 0 and n) read as zero
template <typename T>
__device__ inline T inner(const T* __restrict__ F, int i, int j, int nx, int ny) {
  return (i >= 1 && j >= 1 && i < nx && j < ny) ? F[static_cast<size_t>(j) * nx + i] : T(0);
}

// One axis of a particle's stencil: lowest node b, fraction d, clamped node
// indices, and the shape weights and their slopes (per cell) in precision R,
// zero on the nodes that are not stored.
template <int O, typename R>
struct Axis {
  int b;
  R d;
  int idx[O + 1];
  R w[O + 1], g[O + 1];
};

template <int O, typename R>
__device__ inline Axis<O, R> make_axis(int b, R d, int n) {
  Axis<O, R> A;
  A.b = b;
  A.d = d;
  bool ok[O + 1];
  shape::weights<O>(d, A.w);
  shape::weight_slopes<O>(d, A.g);
  shape::axis_nodes<O>(b, n, A.idx, ok);
#pragma unroll
  for (int q = 0; q <= O; ++q) {
    A.w[q] = ok[q] ? A.w[q] : R(0);
    A.g[q] = ok[q] ? A.g[q] : R(0);
  }
  return A;
}

template <int O, typename T>
__device__ inline Axis<O, T> locate_axis(int c0, T t, int n) {
  int b;
  const T d = shape::locate<O>(c0, t, n, b);
  return make_axis<O, T>(b, d, n);
}

// value and position gradient (per cell) of the shape interpolant of F
template <int O, typename T, typename R>
__device__ inline void interp(const T* __restrict__ F, const Axis<O, R>& X, const Axis<O, R>& Y,
                              int nx, R& v, R& gx, R& gy) {
  v = R(0);
  gx = R(0);
  gy = R(0);
#pragma unroll
  for (int b = 0; b <= O; ++b) {
    const T* row = F + static_cast<size_t>(Y.idx[b]) * nx;
    R rv = R(0), rg = R(0);
#pragma unroll
    for (int a = 0; a <= O; ++a) {
      const R f = static_cast<R>(row[X.idx[a]]);
      rv += X.w[a] * f;
      rg += X.g[a] * f;
    }
    v += Y.w[b] * rv;
    gx += Y.w[b] * rg;
    gy += Y.g[b] * rv;
  }
}

template <typename T>
__device__ inline bool inside_c(int c0, T t, int n) {
  const T fl = floor(t);
  const int c = c0 + static_cast<int>(fl);
  return c >= 0 && (c < n || (c == n && t == fl));
}

}  // namespace

// Transpose of one real (MODE 0) or trial (MODE 1) push from the taped
// state of slice k.  Real: lam_y holds the adjoint of the pushed state on
// entry and that of the slice-k state (push part) on exit; the ring slot of
// f_k is consumed.  Trial: the adjoint of the trial state comes from the
// trial-current adjoints (Jx~ = +lsb_y/2dz, Jy~ = -lsb_x/2dz) gathered at the
// trial position and is added to lam_y.
template <typename T, int MODE, int O, typename Scatter>
__device__ __forceinline__ void adj_push_one(const Geom& g, const Lattice& L,
                                             const AdjPushArgs<T>& a, int I, int J,
                                             Scatter&& scat) {
  const int64_t np = L.np;
  const int64_t p = static_cast<int64_t>(J) * L.nX + I;
  const T w = a.p.w[p];
  if (w == T(0)) return;
  const int nx = g.nx, ny = g.ny;
  const int lpx = 31 - __clz(L.ppc_x), lpy = 31 - __clz(L.ppc_y);
  const int ci0 = I >> lpx, cj0 = J >> lpy;
  const T fx0 = (T(2 * (I & (L.ppc_x - 1)) + 1)) / T(2 * L.ppc_x);
  const T fy0 = (T(2 * (J & (L.ppc_y - 1)) + 1)) / T(2 * L.ppc_y);
  const T inv_hx = static_cast<T>(1.0 / a.hx), inv_hy = static_cast<T>(1.0 / a.hy);
  const T floor_d = static_cast<T>(a.psi_floor);
  const T dz = static_cast<T>(a.dzeta);
  const T b[5] = {T(kAB5[0]), T(kAB5[1]), T(kAB5[2]), T(kAB5[3]), T(kAB5[4])};
  const int k = a.k;
  int slot[5];
  slot[0] = k & 3;                    // f_k (new) ; also f_{k-4}
  for (int m = 1; m <= 4; ++m) slot[m] = (k - m + 8) & 3;   // f_{k-m}
  T y[5] = {a.p.xi_x[p], a.p.xi_y[p], a.p.ux[p], a.p.uy[p], a.p.psi[p]};
  T h[5][5];   // h[m][c] = f_{k-m}[c], m = 1..4
#pragma unroll
  for (int m = 1; m <= 4; ++m)
#pragma unroll
    for (int c = 0; c < 5; ++c) h[m][c] = a.p.hist[(static_cast<size_t>(slot[m]) * 5 + c) * np + p];
  // gather with gradients at the current position
  const Axis<O, T> X = locate_axis<O>(ci0, fx0 + y[0], nx);
  const Axis<O, T> Y = locate_axis<O>(cj0, fy0 + y[1], ny);
  T v[6], gx[6], gy[6];
  const T* F[6] = {a.f.exmby, a.f.eypbx, a.f.ez, a.f.bx, a.f.by, a.f.bz};
#pragma unroll
  for (int c = 0; c < 6; ++c) interp(F[c], X, Y, nx, v[c], gx[c], gy[c]);
  const T e1 = v[0], e2 = v[1], ez = v[2], bx = v[3], by = v[4], bz = v[5];
  const T ux = y[2], uy = y[3];
  const T draw = T(1) + y[4];
  const bool unclamped = !(draw < floor_d);
  const T d = unclamped ? draw : floor_d;
  const T id = T(1) / d;
  const T u2 = T(1) + ux * ux + uy * uy;
  const T gam = (T(1) + ux * ux + uy * uy + d * d) * T(0.5) * id;
  const T G = gam * id;                              // gamma / D
  T f[5];
  f[0] = -ux * id * inv_hx;
  f[1] = -uy * id * inv_hy;
  f[2] = gam * id * e1 + by + bz * uy * id;
  f[3] = gam * id * e2 - bx - bz * ux * id;
  f[4] = (ux * e1 + uy * e2) * id - ez;
  T yn[5];
#pragma unroll
  for (int c = 0; c < 5; ++c)
    yn[c] = y[c] - dz * (b[0] * f[c] + b[1] * h[1][c] + b[2] * h[2][c] + b[3] * h[3][c] + b[4] * h[4][c]);
  const bool moved = inside_c(ci0, fx0 + yn[0], nx) && inside_c(cj0, fy0 + yn[1], ny);
  T* ly = a.lam_y;
  T* lr = a.lam_ring;
  T lnew[5] = {0, 0, 0, 0, 0};
  T lf[5];
  T lf_own[2] = {0, 0};   // trial: lf[2], lf[3] of this iteration's deposit alone
  if (MODE == 0) {
    // adjoint of the pushed state and of the history slot holding f_k
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const T lyk = ly[c * np + p];
      const T lslot = lr[(static_cast<size_t>(slot[0]) * 5 + c) * np + p];
      lnew[c] = moved ? lyk : T(0);
      lf[c] = moved ? (-dz * b[0] * lnew[c] + lslot) : T(0);
      lr[(static_cast<size_t>(slot[0]) * 5 + c) * np + p] = T(0);
    }
  } else {
    if (moved) {
      // deposit transpose of Jx~, Jy~ at the trial state
      const Axis<O, T> TX = locate_axis<O>(ci0, fx0 + yn[0], nx);
      const Axis<O, T> TY = locate_axis<O>(cj0, fy0 + yn[1], ny);
      T gjx, gjx_x, gjx_y, gjy, gjy_x, gjy_y;
      interp(a.lsb_y, TX, TY, nx, gjx, gjx_x, gjx_y);
      interp(a.lsb_x, TX, TY, nx, gjy, gjy_x, gjy_y);
      const T s2 = static_cast<T>(a.inv2dz);
      gjx *= s2; gjx_x *= s2; gjx_y *= s2;
      gjy *= -s2; gjy_x *= -s2; gjy_y *= -s2;
      const T tux = yn[2], tuy = yn[3];
      const T tdraw = T(1) + yn[4];
      const bool tun = !(tdraw < floor_d);
      const T td = tun ? tdraw : floor_d;
      const T tid = T(1) / td;
      const T qn = -w;
      const T vjx = qn * tux * tid, vjy = qn * tuy * tid;
      lnew[0] = vjx * gjx_x + vjy * gjy_x;
      lnew[1] = vjx * gjx_y + vjy * gjy_y;
      lnew[2] = qn * tid * gjx;
      lnew[3] = qn * tid * gjy;
      lnew[4] = tun ? (-qn * tux * tid * tid * gjx - qn * tuy * tid * tid * gjy) : T(0);
    }
    // this iteration's own Bx, By terms use its own deposit adjoint only;
    // the later iterations' sums join everything they share with it
#pragma unroll
    for (int c = 2; c < 4; ++c) lf_own[c - 2] = -dz * b[0] * lnew[c];
    if (a.acc)
#pragma unroll
      for (int c = 0; c < 5; ++c) lnew[c] += a.acc[c * np + p];
#pragma unroll
    for (int c = 0; c < 5; ++c) lf[c] = -dz * b[0] * lnew[c];
  }
  // history adjoints and the identity part of the step
#pragma unroll
  for (int m = 1; m <= 4; ++m)
#pragma unroll
    for (int c = 0; c < 5; ++c)
      if (lnew[c] != T(0)) lr[(static_cast<size_t>(slot[m]) * 5 + c) * np + p] += -dz * b[m] * lnew[c];
  T lam[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) lam[c] = lnew[c];
  // right-hand side transposed
  const T id2 = id * id;
  T lux = -lf[0] * id * inv_hx + lf[2] * (ux * id2) * e1 + lf[3] * ((ux * id2) * e2 - bz * id) + lf[4] * e1 * id;
  T luy = -lf[1] * id * inv_hy + lf[2] * ((uy * id2) * e1 + bz * id) + lf[3] * (uy * id2) * e2 + lf[4] * e2 * id;
  T ld = lf[0] * ux * id2 * inv_hx + lf[1] * uy * id2 * inv_hy +
         lf[2] * (-u2 * id2 * id * e1 - bz * uy * id2) + lf[3] * (-u2 * id2 * id * e2 + bz * ux * id2) +
         lf[4] * (-(ux * e1 + uy * e2) * id2);
  lam[2] += lux;
  lam[3] += luy;
  if (unclamped) lam[4] += ld;
  T lg[6];
  lg[0] = lf[2] * G + lf[4] * ux * id;
  lg[1] = lf[3] * G + lf[4] * uy * id;
  lg[2] = -lf[4];
  lg[3] = MODE == 0 ? -lf[3] : -lf_own[1];
  lg[4] = MODE == 0 ? lf[2] : lf_own[0];
  lg[5] = lf[2] * uy * id - lf[3] * ux * id;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    lam[0] += lg[c] * gx[c];
    lam[1] += lg[c] * gy[c];
    scat(c, X, Y, static_cast<double>(lg[c]));
  }
  if (MODE == 1 && a.acc) {   // the later iterations' own Bx, By position terms
    lam[0] += a.acc[5 * np + p];
    lam[1] += a.acc[6 * np + p];
  }
  if (MODE == 0) {
#pragma unroll
    for (int c = 0; c < 5; ++c) ly[c * np + p] = lam[c];
  } else {
#pragma unroll
    for (int c = 0; c < 5; ++c) ly[c * np + p] += lam[c];
  }
}

// One workgroup per lattice tile (the tiles of the forward push): the
// transposed gathers of the six fields accumulate in FP64 LDS histograms of
// the tile's cells plus a halo and reach the global planes with one atomic
// per non-zero node; stencils outside the histogram go straight to global
// atomics.
template <typename T, int MODE, int O>
__global__ void __launch_bounds__(kBlock) k_adj_push(Geom g, Lattice L, AdjPushArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* tile = reinterpret_cast<double*>(smem_raw);
  const push_detail::TileShape ts = push_detail::tile_shape(L, a.tile_rows, a.tile_halo);
  const int ntile = ts.nw * ts.nh;
  const int nx = g.nx, ny = g.ny;
  for (int e = threadIdx.x; e < 6 * ntile; e += kBlock) tile[e] = 0.0;
  __syncthreads();
  const int I0 = blockIdx.x * ts.tx, J0 = blockIdx.y * ts.ty;
  const int ox = (I0 >> ts.lpx) - ts.halo, oy = (J0 >> ts.lpy) - ts.halo;
  auto scat = [&](int c, const Axis<O, T>& X, const Axis<O, T>& Y, double v) {
    if (v == 0.0) return;
    double sx[O + 1], sy[O + 1];
    shape::weights<O>(static_cast<double>(X.d), sx);
    shape::weights<O>(static_cast<double>(Y.d), sy);
    const int li = X.b - ox, lj = Y.b - oy;
    if (li >= 0 && li + O < ts.nw && lj >= 0 && lj + O < ts.nh) {
      double* t = tile + c * ntile + lj * ts.nw + li;
#pragma unroll
      for (int qb = 0; qb <= O; ++qb)
#pragma unroll
        for (int qa = 0; qa <= O; ++qa) push_detail::lds_add(t + qb * ts.nw + qa, v * (sx[qa] * sy[qb]));
    } else {
#pragma unroll
      for (int qb = 0; qb <= O; ++qb) {
        const int j = Y.b + qb;
#pragma unroll
        for (int qa = 0; qa <= O; ++qa) {
          const int i = X.b + qa;
          if (i >= 1 && i < nx && j >= 1 && j < ny)
            gadd(a.lam_F[c] + static_cast<size_t>(j) * nx + i, v * (sx[qa] * sy[qb]));
        }
      }
    }
  };
  for (int e = threadIdx.x; e < ts.tx * ts.ty; e += kBlock)
    adj_push_one<T, MODE, O>(g, L, a, I0 + e % ts.tx, J0 + e / ts.tx, scat);
  __syncthreads();
  push_detail::flush_tile<6>(a.lam_F, tile, ts, ox, oy, nx, ny);
}

// Transpose of a later predictor-corrector trial push (iteration m >= 1),
// which the forward computes from the slice's trial record: the deposit of
// Jx, Jy at the recorded position with u = u0 - dz b0 (By, -Bx)(x_k).  Its
// Bx, By adjoints are scattered at the slice-k position (the B cotangent of
// iteration m); the adjoints of the recorded quantities, which the first
// trial push's transpose carries back to the state, history and E fields,
// are summed per particle into acc (with the slice-k position terms of this
// iteration's own Bx, By gradients).
template <typename T, int O, typename Scatter>
__device__ __forceinline__ void adj_trial_later_one(const Geom& g, const Lattice& L,
                                                    const AdjPushArgs<T>& a, int I, int J,
                                                    Scatter&& scat) {
  const int64_t np = L.np;
  const int64_t p = static_cast<int64_t>(J) * L.nX + I;
  const T* r = a.rec;
  T* acc = a.acc;
  const bool store = a.acc_mode == 1;
  const T fac = r[4 * np + p];
  if (fac == T(0)) {   // dead, or absorbed by the step: nothing deposited
    if (store)
#pragma unroll
      for (int c = 0; c < 7; ++c) acc[c * np + p] = T(0);
    return;
  }
  const T w = a.p.w[p];
  const T xk = a.p.xi_x[p], ek = a.p.xi_y[p];
  const T xn = r[p], en = r[np + p], cx = r[2 * np + p], cy = r[3 * np + p];
  const T psin = r[5 * np + p];
  const int nx = g.nx, ny = g.ny;
  const int lpx = 31 - __clz(L.ppc_x), lpy = 31 - __clz(L.ppc_y);
  const int ci0 = I >> lpx, cj0 = J >> lpy;
  const T fx0 = (T(2 * (I & (L.ppc_x - 1)) + 1)) / T(2 * L.ppc_x);
  const T fy0 = (T(2 * (J & (L.ppc_y - 1)) + 1)) / T(2 * L.ppc_y);
  const T floor_d = static_cast<T>(a.psi_floor);
  const T dz = static_cast<T>(a.dzeta);
  const T b0 = T(kAB5[0]);
  // this iteration's Bx, By at the slice-k position, with gradients
  const Axis<O, T> X = locate_axis<O>(ci0, fx0 + xk, nx);
  const Axis<O, T> Y = locate_axis<O>(cj0, fy0 + ek, ny);
  T bx, bx_x, bx_y, by, by_x, by_y;
  interp(a.f.bx, X, Y, nx, bx, bx_x, bx_y);
  interp(a.f.by, X, Y, nx, by, by_x, by_y);
  const T kick = dz * b0;
  const T tux = cx - kick * by, tuy = cy + kick * bx;
  const T tdraw = T(1) + psin;
  const bool tun = !(tdraw < floor_d);
  const T tid = T(1) / (tun ? tdraw : floor_d);
  const T qn = -w;
  // deposit transpose of Jx~, Jy~ at the trial position
  const Axis<O, T> TX = locate_axis<O>(ci0, fx0 + xn, nx);
  const Axis<O, T> TY = locate_axis<O>(cj0, fy0 + en, ny);
  T gjx, gjx_x, gjx_y, gjy, gjy_x, gjy_y;
  interp(a.lsb_y, TX, TY, nx, gjx, gjx_x, gjx_y);
  interp(a.lsb_x, TX, TY, nx, gjy, gjy_x, gjy_y);
  const T s2 = static_cast<T>(a.inv2dz);
  gjx *= s2; gjx_x *= s2; gjx_y *= s2;
  gjy *= -s2; gjy_x *= -s2; gjy_y *= -s2;
  const T vjx = qn * tux * tid, vjy = qn * tuy * tid;
  T v[7];
  v[0] = vjx * gjx_x + vjy * gjy_x;
  v[1] = vjx * gjx_y + vjy * gjy_y;
  v[2] = qn * tid * gjx;
  v[3] = qn * tid * gjy;
  v[4] = tun ? (-qn * tux * tid * tid * gjx - qn * tuy * tid * tid * gjy) : T(0);
  // f_x carries +By, f_y -Bx, each times -dz b0 in the step
  const T lgbx = dz * b0 * v[3], lgby = -dz * b0 * v[2];
  scat(0, X, Y, static_cast<double>(lgbx));
  scat(1, X, Y, static_cast<double>(lgby));
  v[5] = lgbx * bx_x + lgby * by_x;
  v[6] = lgbx * bx_y + lgby * by_y;
#pragma unroll
  for (int c = 0; c < 7; ++c) acc[c * np + p] = store ? v[c] : acc[c * np + p] + v[c];
}

// Tiles as in k_adj_push; two LDS histograms (Bx, By adjoints of the
// iteration, lam_F[3] and lam_F[4]).
template <typename T, int O>
__global__ void __launch_bounds__(kBlock) k_adj_trial_later(Geom g, Lattice L, AdjPushArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* tile = reinterpret_cast<double*>(smem_raw);
  const push_detail::TileShape ts = push_detail::tile_shape(L, a.tile_rows, a.tile_halo);
  const int ntile = ts.nw * ts.nh;
  const int nx = g.nx, ny = g.ny;
  for (int e = threadIdx.x; e < 2 * ntile; e += kBlock) tile[e] = 0.0;
  __syncthreads();
  const int I0 = blockIdx.x * ts.tx, J0 = blockIdx.y * ts.ty;
  const int ox = (I0 >> ts.lpx) - ts.halo, oy = (J0 >> ts.lpy) - ts.halo;
  auto scat = [&](int c, const Axis<O, T>& X, const Axis<O, T>& Y, double v) {
    if (v == 0.0) return;
    double sx[O + 1], sy[O + 1];
    shape::weights<O>(static_cast<double>(X.d), sx);
    shape::weights<O>(static_cast<double>(Y.d), sy);
    const int li = X.b - ox, lj = Y.b - oy;
    if (li >= 0 && li + O < ts.nw && lj >= 0 && lj + O < ts.nh) {
      double* t = tile + c * ntile + lj * ts.nw + li;
#pragma unroll
      for (int qb = 0; qb <= O; ++qb)
#pragma unroll
        for (int qa = 0; qa <= O; ++qa) push_detail::lds_add(t + qb * ts.nw + qa, v * (sx[qa] * sy[qb]));
    } else {
#pragma unroll
      for (int qb = 0; qb <= O; ++qb) {
        const int j = Y.b + qb;
#pragma unroll
        for (int qa = 0; qa <= O; ++qa) {
          const int i = X.b + qa;
          if (i >= 1 && i < nx && j >= 1 && j < ny)
            gadd(a.lam_F[3 + c] + static_cast<size_t>(j) * nx + i, v * (sx[qa] * sy[qb]));
        }
      }
    }
  };
  for (int e = threadIdx.x; e < ts.tx * ts.ty; e += kBlock)
    adj_trial_later_one<T, O>(g, L, a, I0 + e % ts.tx, J0 + e / ts.tx, scat);
  __syncthreads();
  push_detail::flush_tile<2>(a.lam_F + 3, tile, ts, ox, oy, nx, ny);
}

// Transpose of the deposit at the slice-k state: gathers the adjoints of
// rho-Jz, Jx, Jy, Jz (FP64 planes) with S and grad S.
template <typename T, int O>
__global__ void __launch_bounds__(kBlock) k_adj_deposit(Geom g, Lattice L, AdjDepArgs<T> a) {
  const int64_t np = L.np;
  const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (p >= np) return;
  const T w = a.p.w[p];
  if (w == T(0)) return;
  const int nx = g.nx, ny = g.ny;
  const int I = static_cast<int>(p % L.nX), J = static_cast<int>(p / L.nX);
  const int lpx = 31 - __clz(L.ppc_x), lpy = 31 - __clz(L.ppc_y);
  const T fx0 = (T(2 * (I & (L.ppc_x - 1)) + 1)) / T(2 * L.ppc_x);
  const T fy0 = (T(2 * (J & (L.ppc_y - 1)) + 1)) / T(2 * L.ppc_y);
  const T xi = a.p.xi_x[p], eta = a.p.xi_y[p], ux = a.p.ux[p], uy = a.p.uy[p], psi = a.p.psi[p];
  int bi, bj;
  const T dx = shape::locate<O>(I >> lpx, fx0 + xi, nx, bi);
  const T dy = shape::locate<O>(J >> lpy, fy0 + eta, ny, bj);
  const Axis<O, double> X = make_axis<O, double>(bi, static_cast<double>(dx), nx);
  const Axis<O, double> Y = make_axis<O, double>(bj, static_cast<double>(dy), ny);
  const T floor_d = static_cast<T>(a.psi_floor);
  const T draw = T(1) + psi;
  const bool un = !(draw < floor_d);
  const T d = un ? draw : floor_d;
  const T id = T(1) / d;
  const T u2 = T(1) + ux * ux + uy * uy;
  const T qn = -w;
  const T val[4] = {qn, qn * ux * id, qn * uy * id, qn * (u2 * T(0.5) * id * id - T(0.5))};
  const T dux[4] = {T(0), qn * id, T(0), qn * ux * id * id};
  const T duy[4] = {T(0), T(0), qn * id, qn * uy * id * id};
  const T dd[4] = {T(0), -qn * ux * id * id, -qn * uy * id * id, -qn * u2 * id * id * id};
  T l[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double v, gxv, gyv;
    interp(a.lam_dep[c], X, Y, nx, v, gxv, gyv);
    l[0] += val[c] * static_cast<T>(gxv);
    l[1] += val[c] * static_cast<T>(gyv);
    l[2] += dux[c] * static_cast<T>(v);
    l[3] += duy[c] * static_cast<T>(v);
    if (un) l[4] += dd[c] * static_cast<T>(v);
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) a.lam_y[c * np + p] += l[c];
}

// ------------------------------------------------------------------ grid side

// out[c] = cotangent of field c at slice k (node layout, T; boundary nodes
// dropped) + extra[c] (FP64 stored layout); both may be null.  Also clears
// the planes zero[0..2] (the per-slice accumulators).
template <typename T>
__global__ void k_adj_seed(Geom g, AdjSeedArgs<T> a) {
  const size_t n = static_cast<size_t>(g.nx) * g.ny;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n; e += stride) {
    const int i = static_cast<int>(e % g.nx), j = static_cast<int>(e / g.nx);
    const bool interior = i > 0 && j > 0;
    const size_t nodes = static_cast<size_t>(j) * (g.nx + 1) + i;
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      double v = 0.0;
      if (interior && a.cot[c]) v = static_cast<double>(a.cot[c][nodes]);
      if (a.extra[c]) v += a.extra[c][e];
      a.out[c][e] = v;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (a.zero[c]) a.zero[c][e] = 0.0;
  }
}

// predictor-corrector step m, grid part: from the solved adjoint sources
// lsb = (lap - s)^-1 lam_B^{m+1}:  lam_Jz += d_y lsb_x - d_x lsb_y,
// lam_Jprev += (-lsb_y, lsb_x) / 2dz, lam_B^m = -s lsb (the trial kernel then
// adds its gather transpose).
template <typename T>
__global__ void k_adj_pc_grid(Geom g, AdjPCGridArgs<T> a) {
  const int nx = g.nx, ny = g.ny;
  const size_t n = static_cast<size_t>(nx) * ny;
  const double ihx = 0.5 / g.hx, ihy = 0.5 / g.hy;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n; e += stride) {
    const int i = static_cast<int>(e % nx), j = static_cast<int>(e / nx);
    const double sx = a.lsb_x[e], sy = a.lsb_y[e];
    double djz = 0.0;
    if (i > 0 && j > 0) {
      const double sx_n = inner(a.lsb_x, i, j + 1, nx, ny), sx_s = inner(a.lsb_x, i, j - 1, nx, ny);
      const double sy_e = inner(a.lsb_y, i + 1, j, nx, ny), sy_w = inner(a.lsb_y, i - 1, j, nx, ny);
      djz = (sx_n - sx_s) * ihy - (sy_e - sy_w) * ihx;
    }
    a.lam_jz[e] += djz;
    a.jp_x[e] += -sy * a.inv2dz;
    a.jp_y[e] += sx * a.inv2dz;
    a.lam_bx[e] = -a.shift * sx;
    a.lam_by[e] = -a.shift * sy;
  }
}

// initial guess B^0 = 2 B_{k-1} - B_{k-2}, transposed; the adjoint of B_{k-1}
// also collects what slice k+1 handed to B_{k-1} (its B_{k-2})
__global__ void k_adj_guess(size_t n, const double* lam_b0x, const double* lam_b0y,
                            const double* carry_b2x, const double* carry_b2y, double* b1x,
                            double* b1y, double* b2x, double* b2y) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n; e += stride) {
    b1x[e] = carry_b2x[e] + 2.0 * lam_b0x[e];
    b1y[e] = carry_b2y[e] + 2.0 * lam_b0y[e];
    b2x[e] = -lam_b0x[e];
    b2y[e] = -lam_b0y[e];
  }
}

// adjoints of the deposit channels of slice k from the solved adjoint
// sources, and the beam-parameter gradient of slice k:
//   lam_R = -lpsi,  lam_Jx = carry_jx - d_x lez - d_y lbz,
//   lam_Jy = carry_jy - d_y lez + d_x lbz,  lam_Jz as accumulated;
//   dL/da_k = -<lam_Jz, G>,  dL/dsigma += -a_k <lam_Jz, dG/dsigma>.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_adj_dep_grid(Geom g, AdjDepGridArgs<T> a) {
  const int nx = g.nx, ny = g.ny;
  const size_t n = static_cast<size_t>(nx) * ny;
  const double ihx = 0.5 / g.hx, ihy = 0.5 / g.hy;
  double s_amp = 0.0, s_sx = 0.0, s_sy = 0.0;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n; e += stride) {
    const int i = static_cast<int>(e % nx), j = static_cast<int>(e / nx);
    double r = 0.0, jx = a.carry_jx[e], jy = a.carry_jy[e];
    if (i > 0 && j > 0) {
      r = -static_cast<double>(a.lpsi[e]);
      const double ez_e = inner(a.lez, i + 1, j, nx, ny), ez_w = inner(a.lez, i - 1, j, nx, ny);
      const double ez_n = inner(a.lez, i, j + 1, nx, ny), ez_s = inner(a.lez, i, j - 1, nx, ny);
      const double bz_e = inner(a.lbz, i + 1, j, nx, ny), bz_w = inner(a.lbz, i - 1, j, nx, ny);
      const double bz_n = inner(a.lbz, i, j + 1, nx, ny), bz_s = inner(a.lbz, i, j - 1, nx, ny);
      jx += -(ez_e - ez_w) * ihx - (bz_n - bz_s) * ihy;
      jy += -(ez_n - ez_s) * ihy + (bz_e - bz_w) * ihx;
      const double lz = a.lam_jz[e];
      s_amp += lz * a.bgx[i] * a.bgy[j];
      s_sx += lz * a.dbgx[i] * a.bgy[j];
      s_sy += lz * a.bgx[i] * a.dbgy[j];
    } else {
      jx = jy = 0.0;
    }
    a.lam_r[e] = r;
    a.lam_jx[e] = jx;
    a.lam_jy[e] = jy;
  }
  __shared__ double red[3][kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) {
    s_amp += __shfl_down(s_amp, off, 64);
    s_sx += __shfl_down(s_sx, off, 64);
    s_sy += __shfl_down(s_sy, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = s_amp;
    red[1][wave] = s_sx;
    red[2][wave] = s_sy;
  }
  __syncthreads();
  if (threadIdx.x == 0 && a.grad_amp) {
    double t0 = 0, t1 = 0, t2 = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      t0 += red[0][w];
      t1 += red[1][w];
      t2 += red[2][w];
    }
    gadd(a.grad_amp + a.k, -t0);
    gadd(a.grad_sigma, -a.amp * t1);
    gadd(a.grad_sigma + 1, -a.amp * t2);
  }
}

// sources of up to three adjoint solves:
//   out[q] = c0[q] * P0[q] + c1[q] * d_x P1[q] + c2[q] * d_y P2[q]
// (FP64 stored planes, any may be null; zero on the Dirichlet nodes), cast to T
template <typename T>
__global__ void k_adj_source(Geom g, AdjSrcArgs<T> a) {
  const int nx = g.nx, ny = g.ny;
  const size_t n = static_cast<size_t>(nx) * ny;
  const double ihx = 0.5 / g.hx, ihy = 0.5 / g.hy;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n; e += stride) {
    const int i = static_cast<int>(e % nx), j = static_cast<int>(e / nx);
    for (int q = 0; q < a.count; ++q) {
      double s = 0.0;
      if (i > 0 && j > 0) {
        if (a.p0[q]) s += a.c0[q] * a.p0[q][e];
        if (a.p1[q]) s += a.c1[q] * (inner(a.p1[q], i + 1, j, nx, ny) - inner(a.p1[q], i - 1, j, nx, ny)) * ihx;
        if (a.p2[q]) s += a.c2[q] * (inner(a.p2[q], i, j + 1, nx, ny) - inner(a.p2[q], i, j - 1, nx, ny)) * ihy;
      }
      a.out[q][e] = static_cast<T>(s);
    }
  }
}

// sum_F <W_F(k), F_k> over the given fields into *loss (FP64)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_loss(Geom g, LossArgs<T> a) {
  const size_t n = static_cast<size_t>(g.nx) * g.ny;
  double s = 0.0;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n; e += stride) {
    const int i = static_cast<int>(e % g.nx), j = static_cast<int>(e / g.nx);
    if (i == 0 || j == 0) continue;
    const size_t nodes = static_cast<size_t>(j) * (g.nx + 1) + i;
#pragma unroll
    for (int c = 0; c < 7; ++c)
      if (a.cot[c] && a.field[c])
        s += static_cast<double>(a.cot[c][nodes]) * static_cast<double>(a.field[c][e]);
  }
  __shared__ double red[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    gadd(a.loss, t);
  }
}

template <typename T>
__global__ void k_copy_particles(Lattice L, Particles<T> src, Particles<T> dst, int k, T dz) {
  const size_t np = static_cast<size_t>(L.np);
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  // history slots of f_{k-1}, ..., f_{k-4}
  const int s1 = (k + 3) & 3, s2 = (k + 2) & 3, s3 = (k + 1) & 3, s4 = k & 3;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < np; i += stride) {
    T y[5] = {src.xi_x[i], src.xi_y[i], src.ux[i], src.uy[i], src.psi[i]};
    dst.xi_x[i] = y[0];
    dst.xi_y[i] = y[1];
    dst.ux[i] = y[2];
    dst.uy[i] = y[3];
    dst.psi[i] = y[4];
    dst.w[i] = src.w[i];
#pragma unroll
    for (int c = 0; c < 20; ++c) dst.hist[c * np + i] = src.hist[c * np + i];
    if (dst.pab) {
      const T* h = src.hist;
#pragma unroll
      for (int c = 0; c < 5; ++c)
        dst.pab[c * np + i] = ab5_history(y[c], h[(s1 * 5 + c) * np + i], h[(s2 * 5 + c) * np + i],
                                          h[(s3 * 5 + c) * np + i], h[(s4 * 5 + c) * np + i], dz);
    }
  }
}

template <typename T, typename U>
__global__ void k_copy_planes(size_t n, int count, CopyPlanes<T, U> c) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n; e += stride)
    for (int q = 0; q < count; ++q) c.dst[q][e] = static_cast<U>(c.src[q][e]);
}

// ------------------------------------------------------------------ launchers
namespace {
dim3 g1(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b == 0) b = 1;
  return dim3(static_cast<unsigned>(b));
}
dim3 gp(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return dim3(static_cast<unsigned>(b));
}

// the adjoint needs a shape with a derivative: orders 1-3
template <typename F>
void with_adj_order(int order, F&& f) {
  switch (order) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    default: throw std::invalid_argument("the adjoint needs a shape order of 1, 2 or 3");
  }
}
}  // namespace

template <typename T>
void launch_adj_push(const Geom& g, const Lattice& L, const AdjPushArgs<T>& a, bool trial,
                     hipStream_t st) {
  const push_detail::TileShape ts = push_detail::tile_shape(L, a.tile_rows, a.tile_halo);
  const size_t lds = static_cast<size_t>(6) * ts.nw * ts.nh * sizeof(double);
  if (lds > 160 * 1024) throw std::invalid_argument("adjoint push histogram exceeds the LDS");
  const dim3 grid(L.nX / ts.tx, L.nY / ts.ty);
  with_adj_order(g.order, [&](auto order) {
    constexpr int O = decltype(order)::value;
    const void* fn = trial ? reinterpret_cast<const void*>(&k_adj_push<T, 1, O>)
                           : reinterpret_cast<const void*>(&k_adj_push<T, 0, O>);
    if (lds > 65536)
      QSP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    if (trial)
      hipLaunchKernelGGL((k_adj_push<T, 1, O>), grid, dim3(kBlock), lds, st, g, L, a);
    else
      hipLaunchKernelGGL((k_adj_push<T, 0, O>), grid, dim3(kBlock), lds, st, g, L, a);
  });
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_adj_trial_later(const Geom& g, const Lattice& L, const AdjPushArgs<T>& a,
                            hipStream_t st) {
  if (!a.rec || !a.acc || (a.acc_mode != 1 && a.acc_mode != 2))
    throw std::invalid_argument("a later trial push transpose needs the record and the sums");
  const push_detail::TileShape ts = push_detail::tile_shape(L, a.tile_rows, a.tile_halo);
  const size_t lds = static_cast<size_t>(2) * ts.nw * ts.nh * sizeof(double);
  if (lds > 160 * 1024) throw std::invalid_argument("adjoint push histogram exceeds the LDS");
  const dim3 grid(L.nX / ts.tx, L.nY / ts.ty);
  with_adj_order(g.order, [&](auto order) {
    constexpr int O = decltype(order)::value;
    if (lds > 65536)
      QSP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adj_trial_later<T, O>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    hipLaunchKernelGGL((k_adj_trial_later<T, O>), grid, dim3(kBlock), lds, st, g, L, a);
  });
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_adj_deposit(const Geom& g, const Lattice& L, const AdjDepArgs<T>& a, hipStream_t st) {
  with_adj_order(g.order, [&](auto order) {
    hipLaunchKernelGGL((k_adj_deposit<T, decltype(order)::value>), gp(L.np), dim3(kBlock), 0, st,
                       g, L, a);
  });
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_adj_seed(const Geom& g, const AdjSeedArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_seed<T>, g1(static_cast<size_t>(g.nx) * g.ny), dim3(kBlock), 0, st, g, a);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_adj_pc_grid(const Geom& g, const AdjPCGridArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_pc_grid<T>, g1(static_cast<size_t>(g.nx) * g.ny), dim3(kBlock), 0, st, g,
                     a);
  QSP_LAUNCH_CHECK();
}

void launch_adj_guess(size_t n, const double* lam_b0x, const double* lam_b0y, const double* c2x,
                      const double* c2y, double* b1x, double* b1y, double* b2x, double* b2y,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_adj_guess, g1(n), dim3(kBlock), 0, st, n, lam_b0x, lam_b0y, c2x, c2y, b1x, b1y,
                     b2x, b2y);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_adj_dep_grid(const Geom& g, const AdjDepGridArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_dep_grid<T>, g1(static_cast<size_t>(g.nx) * g.ny), dim3(kBlock), 0, st, g,
                     a);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_adj_source(const Geom& g, const AdjSrcArgs<T>& a, hipStream_t st) {
  if (a.count < 1 || a.count > 3) throw std::invalid_argument("adjoint source: 1..3 planes");
  hipLaunchKernelGGL(k_adj_source<T>, g1(static_cast<size_t>(g.nx) * g.ny), dim3(kBlock), 0, st, g, a);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_loss(const Geom& g, const LossArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL(k_loss<T>, g1(static_cast<size_t>(g.nx) * g.ny), dim3(kBlock), 0, st, g, a);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_copy_particles(const Lattice& L, const Particles<T>& src, const Particles<T>& dst,
                           int k, double dzeta, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_particles<T>, g1(static_cast<size_t>(L.np)), dim3(kBlock), 0, st, L, src,
                     dst, k, static_cast<T>(dzeta));
  QSP_LAUNCH_CHECK();
}

template <typename T, typename U>
void launch_copy_planes(size_t n, int count, const CopyPlanes<T, U>& c, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL((k_copy_planes<T, U>), g1(n), dim3(kBlock), 0, st, n, count, c);
  QSP_LAUNCH_CHECK();
}

#define QSP_INST(T)                                                                             \
  template void launch_adj_push<T>(const Geom&, const Lattice&, const AdjPushArgs<T>&, bool,    \
                                   hipStream_t);                                               \
  template void launch_adj_trial_later<T>(const Geom&, const Lattice&, const AdjPushArgs<T>&,   \
                                          hipStream_t);                                        \
  template void launch_adj_deposit<T>(const Geom&, const Lattice&, const AdjDepArgs<T>&,        \
                                      hipStream_t);                                            \
  template void launch_adj_seed<T>(const Geom&, const AdjSeedArgs<T>&, hipStream_t);            \
  template void launch_adj_pc_grid<T>(const Geom&, const AdjPCGridArgs<T>&, hipStream_t);       \
  template void launch_adj_dep_grid<T>(const Geom&, const AdjDepGridArgs<T>&, hipStream_t);     \
  template void launch_adj_source<T>(const Geom&, const AdjSrcArgs<T>&, hipStream_t);           \
  template void launch_loss<T>(const Geom&, const LossArgs<T>&, hipStream_t);                   \
  template void launch_copy_particles<T>(const Lattice&, const Particles<T>&,                   \
                                         const Particles<T>&, int, double, hipStream_t);        \
  template void launch_copy_planes<T, T>(size_t, int, const CopyPlanes<T, T>&, hipStream_t);
QSP_INST(float)
QSP_INST(double)
#undef QSP_INST

}  // namespace qsp
