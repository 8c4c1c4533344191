// Device-side body of the fused plasma gather + Adams-Bashforth push +
// deposit (HiPACE++, arXiv:2109.10277, Sec. III.B: plasma pusher equations;
// deposition zeroth order in zeta, transverse shape of order 0-3).
//
// Particles are stored SoA in lattice order and keep their lattice site for
// life; positions are stored as displacements from that site (in cells) so
// that small displacements keep full precision.  A workgroup owns a tile of
// lattice sites; its particles deposit into FP64 histograms in LDS covering
// the tile's cells plus a halo, which are then added to the global FP64
// deposit arrays: the nodes of the tile's own cells with plain stores, the
// halo nodes with one atomic per non-zero node into shared planes (DepOut).
// Particles that have left the tile+halo fall back to global FP64 atomics.
#pragma once

#include "common.hpp"
#include "kernels.hpp"
#include "shape.hpp"

namespace qsp {
namespace push_detail {

struct TileShape {
  int tx, ty;      // lattice sites per tile
  int lpx, lpy;    // log2 ppc
  int nw, nh;      // LDS node tile (cells + 1 + 2 halo)
  int halo;        // cells around the tile's own cells covered in LDS
};

__host__ __device__ inline int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

__host__ __device__ inline TileShape tile_shape(const Lattice& L, int rows, int halo) {
  TileShape t;
  t.halo = halo;
  t.tx = L.nX < 64 ? L.nX : 64;
  t.ty = L.nY < rows ? L.nY : rows;
  t.lpx = ilog2(L.ppc_x);
  t.lpy = ilog2(L.ppc_y);
  t.nw = (t.tx >> t.lpx) + 1 + 2 * halo;
  t.nh = (t.ty >> t.lpy) + 1 + 2 * halo;
  return t;
}

// base[i] with the byte offset formed in 32 bits (the caller guarantees
// i * sizeof(T) < 2^32), so that a uniform base loads through one VGPR of
// offset instead of a 64-bit address per lane
template <typename T>
__device__ __forceinline__ T load_at(const T* base, unsigned int i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                     i * static_cast<unsigned int>(sizeof(T)));
}

template <typename T>
__device__ inline bool inside(int c0, T t, int n) {
  const T fl = floor(t);
  const int c = c0 + static_cast<int>(fl);
  return c >= 0 && (c < n || (c == n && t == fl));
}

// CIC interpolation in cell (i, j), 0 <= i < nx, 0 <= j < ny; the upper
// Dirichlet nodes (index n, not stored) are zero.  All four loads are
// unconditional (clamped indices) so that they issue together.
template <typename T>
__device__ inline T gather(const T* __restrict__ F, int i, int j, T w00, T w10, T w01, T w11,
                           int nx, int ny) {
  const bool ie = i + 1 < nx, jn = j + 1 < ny;
  const int i1 = ie ? i + 1 : i, j1 = jn ? j + 1 : j;
  const T f00 = F[j * nx + i], f10 = F[j * nx + i1], f01 = F[j1 * nx + i], f11 = F[j1 * nx + i1];
  return w00 * f00 + w10 * (ie ? f10 : T(0)) + w01 * (jn ? f01 : T(0)) +
         w11 * ((ie && jn) ? f11 : T(0));
}

__device__ inline void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline void global_add(double* p, double v) { unsafeAtomicAdd(p, v); }

// Adds the nch channels of a tile histogram (nw x nh nodes starting at
// global node (ox, oy), channel c at tile + c * nw * nh) to the global FP64
// planes ch[c]: one atomic per stored, non-zero node.  Nodes are walked in
// row-major order, kBlock at a time, with a running (row, column) pair
// instead of divisions, and the channel loop is unrolled so that each
// plane's address is a compile-time argument offset: no load, and so no
// wait on the atomics already in flight, precedes an atomic.
template <int nch>
__device__ __forceinline__ void flush_tile(double* const* ch, const double* tile,
                                           const TileShape& ts, int ox, int oy, int nx, int ny) {
  const int ntile = ts.nw * ts.nh;
  const int step_r = kBlock / ts.nw, step_c = kBlock % ts.nw;
  int r = threadIdx.x / ts.nw, cl = threadIdx.x % ts.nw;
  for (int l = threadIdx.x; l < ntile; l += kBlock) {
    const int gi = ox + cl, gj = oy + r;
    if (gi >= 1 && gi < nx && gj >= 1 && gj < ny) {
      const size_t o = static_cast<size_t>(gj) * nx + gi;
      double val[nch];
#pragma unroll
      for (int c = 0; c < nch; ++c) val[c] = tile[c * ntile + l];
#pragma unroll
      for (int c = 0; c < nch; ++c)
        if (val[c] != 0.0) global_add(ch[c] + o, val[c]);
    }
    r += step_r;
    cl += step_c;
    if (cl >= ts.nw) {
      cl -= ts.nw;
      ++r;
    }
  }
}

// Owner form of flush_tile: the nodes of the tile's own cells (local
// columns halo .. halo + tx/ppc_x - 1, rows likewise) are stored into ch[c],
// zeros included; the other non-zero nodes are added to sh[c] with atomics.
template <int nch>
__device__ __forceinline__ void flush_tile_owned(double* const* ch, double* const* sh,
                                                 const double* tile, const TileShape& ts, int ox,
                                                 int oy, int nx, int ny) {
  const int ntile = ts.nw * ts.nh;
  const unsigned int ocx = static_cast<unsigned int>(ts.tx >> ts.lpx);
  const unsigned int ocy = static_cast<unsigned int>(ts.ty >> ts.lpy);
  const int step_r = kBlock / ts.nw, step_c = kBlock % ts.nw;
  int r = threadIdx.x / ts.nw, cl = threadIdx.x % ts.nw;
  for (int l = threadIdx.x; l < ntile; l += kBlock) {
    const int gi = ox + cl, gj = oy + r;
    if (gi >= 1 && gi < nx && gj >= 1 && gj < ny) {
      const size_t o = static_cast<size_t>(gj) * nx + gi;
      const bool own = static_cast<unsigned int>(cl - ts.halo) < ocx &&
                       static_cast<unsigned int>(r - ts.halo) < ocy;
      double val[nch];
#pragma unroll
      for (int c = 0; c < nch; ++c) val[c] = tile[c * ntile + l];
#pragma unroll
      for (int c = 0; c < nch; ++c) {
        if (own)
          ch[c][o] = val[c];
        else if (val[c] != 0.0)
          global_add(sh[c] + o, val[c]);
      }
    }
    r += step_r;
    cl += step_c;
    if (cl >= ts.nw) {
      cl -= ts.nw;
      ++r;
    }
  }
}

__device__ inline unsigned long long block_sum(unsigned int v, unsigned int* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  unsigned long long s = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
  return s;
}

// Deposit of one particle: nch values v at offset (xi, eta) from its
// lattice cell origin (ci0 + fx0, cj0 + fy0) into the tile histogram, or
// straight to the global planes (the shared ones for an owner flush) when
// the stencil leaves the tile (counted in nglob).  A particle that is not
// live deposits zeros into the histogram and nothing outside it.
template <typename T, int O, int nch>
__device__ __forceinline__ void deposit_particle(const DepOut& dep, double* tile, const TileShape& ts,
                                                 int ox, int oy, int nx, int ny, bool tiled,
                                                 bool owner, int ci0,
                                                 int cj0, T fx0, T fy0, T xi, T eta,
                                                 const double (&v)[4], unsigned int& nglob,
                                                 bool live = true) {
  const int ntile = ts.nw * ts.nh;
  int bi, bj;
  const T dx = shape::locate<O>(ci0, fx0 + xi, nx, bi);
  const T dy = shape::locate<O>(cj0, fy0 + eta, ny, bj);
  double sx[O + 1], sy[O + 1];
  shape::weights<O>(static_cast<double>(dx), sx);
  shape::weights<O>(static_cast<double>(dy), sy);
  const int li = bi - ox, lj = bj - oy;
  if (tiled && li >= 0 && li + O < ts.nw && lj >= 0 && lj + O < ts.nh) {
    const int base = lj * ts.nw + li;
#pragma unroll
    for (int c = 0; c < nch; ++c) {
      double* t = tile + c * ntile + base;
#pragma unroll
      for (int qb = 0; qb <= O; ++qb)
#pragma unroll
        for (int qa = 0; qa <= O; ++qa) lds_add(t + qb * ts.nw + qa, v[c] * (sx[qa] * sy[qb]));
    }
  } else if (live) {
    if (tiled) ++nglob;
#pragma unroll
    for (int qb = 0; qb <= O; ++qb) {
      const int gj = bj + qb;
#pragma unroll
      for (int qa = 0; qa <= O; ++qa) {
        const int gi = bi + qa;
        if (gi < 1 || gi >= nx || gj < 1 || gj >= ny) continue;
        const size_t o = static_cast<size_t>(gj) * nx + gi;
        const double s = sx[qa] * sy[qb];
#pragma unroll
        for (int c = 0; c < nch; ++c) global_add((owner ? dep.sh[c] : dep.ch[c]) + o, v[c] * s);
      }
    }
  }
}

// Bx, By at displacement (xk, ek) from the lattice cell origin
// (ci0 + fx0, cj0 + fy0), shape order O (indices clamped: always in bounds).
template <typename T, int O>
__device__ __forceinline__ void gather_bxby(const SliceFields<T>& f, int ci0, int cj0, T fx0, T fy0,
                                            T xk, T ek, int nx, int ny, T& bx, T& by) {
  if constexpr (O == 1) {
    int ci, cj;
    const T fx = shape::locate<1>(ci0, fx0 + xk, nx, ci);
    const T fy = shape::locate<1>(cj0, fy0 + ek, ny, cj);
    const T w00 = (T(1) - fx) * (T(1) - fy), w10 = fx * (T(1) - fy);
    const T w01 = (T(1) - fx) * fy, w11 = fx * fy;
    bx = gather(f.bx, ci, cj, w00, w10, w01, w11, nx, ny);
    by = gather(f.by, ci, cj, w00, w10, w01, w11, nx, ny);
  } else {
    int bi, bj;
    const T dx = shape::locate<O>(ci0, fx0 + xk, nx, bi);
    const T dy = shape::locate<O>(cj0, fy0 + ek, ny, bj);
    T wx[O + 1], wy[O + 1];
    int ix[O + 1], iy[O + 1];
    bool okx[O + 1], oky[O + 1];
    shape::weights<O>(dx, wx);
    shape::weights<O>(dy, wy);
    shape::axis_nodes<O>(bi, nx, ix, okx);
    shape::axis_nodes<O>(bj, ny, iy, oky);
#pragma unroll
    for (int q = 0; q <= O; ++q) {
      wx[q] = okx[q] ? wx[q] : T(0);
      wy[q] = oky[q] ? wy[q] : T(0);
    }
    bx = shape::interp<O>(f.bx, ix, iy, wx, wy, nx);
    by = shape::interp<O>(f.by, ix, iy, wx, wy, nx);
  }
}

// Trial push of a later predictor-corrector iteration for the particles of
// the tile at lattice site (I0, J0).  Between iterations only Bx, By
// change, and they enter the push as a kick -dz b0 (By, -Bx) on the
// momentum: the new position, Psi and the rest of the momentum come from the
// slice's first trial push (the record), and Bx, By are gathered at the
// slice-k position as there.  A thread takes kLaterBatch particles at a
// time (FP32 linear shape; one otherwise, whose registers two would crowd)
// and issues all their loads, then all their gathers, before its first
// deposit; a particle without deposit (record factor 0) adds zeros, so that
// nothing waits on the factor.
constexpr int kLaterBatch = 2;

template <typename T, int O, int nch>
__device__ __forceinline__ void trial_later_particles(const Lattice& L, const PushArgs<T>& a,
                                                      double* tile, const TileShape& ts, int I0,
                                                      int J0, int ox, int oy, int nx, int ny,
                                                      bool tiled, bool owner, unsigned int& nglob) {
  constexpr int U = sizeof(T) == 4 && O == 1 ? kLaterBatch : 1;
  const size_t np = static_cast<size_t>(L.np);
  const T* r = a.rec;
  const T kick = static_cast<T>(a.dzeta) * T(kAB5[0]);
  const int ntot = ts.tx * ts.ty;
  for (int e0 = 0; e0 < ntot; e0 += U * kBlock) {
    T fac[U], xk[U], ek[U], xn[U], en[U], cx[U], cy[U], bx[U], by[U];
    int ci0[U], cj0[U];
    T fx0[U], fy0[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kBlock + static_cast<int>(threadIdx.x);
      const int ec = e < ntot ? e : 0;   // a missing particle reads the tile's first
      const int I = I0 + ec % ts.tx, J = J0 + ec / ts.tx;
      // 32-bit offsets from uniform plane bases (the launch checks that a
      // particle plane is below 4 GiB)
      const unsigned int p = static_cast<unsigned int>(J) * static_cast<unsigned int>(L.nX) +
                             static_cast<unsigned int>(I);
      fac[u] = load_at(r + 4 * np, p);
      xk[u] = load_at(a.p.xi_x, p);
      ek[u] = load_at(a.p.xi_y, p);
      xn[u] = load_at(r, p);
      en[u] = load_at(r + np, p);
      cx[u] = load_at(r + 2 * np, p);
      cy[u] = load_at(r + 3 * np, p);
      ci0[u] = I >> ts.lpx;
      cj0[u] = J >> ts.lpy;
      fx0[u] = (T(2 * (I & (L.ppc_x - 1)) + 1)) / T(2 * L.ppc_x);
      fy0[u] = (T(2 * (J & (L.ppc_y - 1)) + 1)) / T(2 * L.ppc_y);
    }
    // keep the scheduler from moving a later particle's loads behind an
    // earlier one's gather (the wait for a load also waits for every load
    // issued before it)
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (O == 1) {
      // the gather of every particle of the batch: addresses and weights,
      // then all loads, then the sums (the same sums as gather())
      unsigned int off[U][4];
      T wt[U][4];
      bool ie[U], jn[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int ci, cj;
        const T fx = shape::locate<1>(ci0[u], fx0[u] + xk[u], nx, ci);
        const T fy = shape::locate<1>(cj0[u], fy0[u] + ek[u], ny, cj);
        wt[u][0] = (T(1) - fx) * (T(1) - fy);
        wt[u][1] = fx * (T(1) - fy);
        wt[u][2] = (T(1) - fx) * fy;
        wt[u][3] = fx * fy;
        ie[u] = ci + 1 < nx;
        jn[u] = cj + 1 < ny;
        const unsigned int r0 = static_cast<unsigned int>(cj * nx);
        const unsigned int r1 = static_cast<unsigned int>((jn[u] ? cj + 1 : cj) * nx);
        const unsigned int c0 = static_cast<unsigned int>(ci);
        const unsigned int c1 = static_cast<unsigned int>(ie[u] ? ci + 1 : ci);
        off[u][0] = r0 + c0;
        off[u][1] = r0 + c1;
        off[u][2] = r1 + c0;
        off[u][3] = r1 + c1;
      }
      T gx[U][4], gy[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          gx[u][q] = load_at(a.f.bx, off[u][q]);
          gy[u][q] = load_at(a.f.by, off[u][q]);
        }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool e1 = ie[u], n1 = jn[u], en1 = ie[u] && jn[u];
        bx[u] = wt[u][0] * gx[u][0] + wt[u][1] * (e1 ? gx[u][1] : T(0)) +
                wt[u][2] * (n1 ? gx[u][2] : T(0)) + wt[u][3] * (en1 ? gx[u][3] : T(0));
        by[u] = wt[u][0] * gy[u][0] + wt[u][1] * (e1 ? gy[u][1] : T(0)) +
                wt[u][2] * (n1 ? gy[u][2] : T(0)) + wt[u][3] * (en1 ? gy[u][3] : T(0));
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u)
        gather_bxby<T, O>(a.f, ci0[u], cj0[u], fx0[u], fy0[u], xk[u], ek[u], nx, ny, bx[u],
                          by[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (e0 + u * kBlock + static_cast<int>(threadIdx.x) >= ntot) continue;
      const bool live = fac[u] != T(0);   // selects, not branches
      const double v[4] = {live ? static_cast<double>(fac[u] * (cx[u] - kick * by[u])) : 0.0,
                           live ? static_cast<double>(fac[u] * (cy[u] + kick * bx[u])) : 0.0, 0.0,
                           0.0};
      deposit_particle<T, O, nch>(a.dep, tile, ts, ox, oy, nx, ny, tiled, owner, ci0[u], cj0[u],
                                  fx0[u], fy0[u], xn[u], en[u], v, nglob, live);
    }
  }
}

// Gather, push and deposit of the particles of lattice tile (tbx, tby) by
// one workgroup with the transverse shape of order O; `tile` is the
// workgroup's LDS histogram (nch channels of tile_shape's nw x nh nodes).
// Safe to call repeatedly from one workgroup.  The linear shape keeps a
// gather of its own (four weights, value selects at the upper edge), which
// the compiler allocates in fewer registers than the generic stencil.
template <typename T, int MODE, int O, bool TAPE = false>
__device__ __forceinline__ void push_tile(const Geom& g, const Lattice& L, const PushArgs<T>& a,
                                          DevCounters* ctr, int tbx, int tby, double* tile) {
  // channels: trial push Jx, Jy; otherwise rho - Jz, Jx, Jy, Jz
  constexpr bool trial = MODE == kPushTrial || MODE == kTrialLater;
  constexpr int nch = trial ? 2 : 4;
  __shared__ unsigned int red[kBlock / 64];
  const TileShape ts = tile_shape(L, a.tile_rows, a.tile_halo);
  const int ntile = ts.nw * ts.nh;
  const bool tiled = a.tiled != 0;
  const bool owner = tiled && a.dep.sh[0] != nullptr;
  if (tiled) {
    __syncthreads();   // a previous tile's flush has read the histogram
    for (int e = threadIdx.x; e < nch * ntile; e += kBlock) tile[e] = 0.0;
    __syncthreads();
  }
  const int I0 = tbx * ts.tx, J0 = tby * ts.ty;
  const int ox = (I0 >> ts.lpx) - ts.halo, oy = (J0 >> ts.lpy) - ts.halo;
  const int nx = g.nx, ny = g.ny;
  const T inv_hx = static_cast<T>(1.0 / a.hx), inv_hy = static_cast<T>(1.0 / a.hy);
  const T floor_d = static_cast<T>(a.psi_floor);
  const T dz = static_cast<T>(a.dzeta);
  const T b0 = T(kAB5[0]);
  const size_t np = static_cast<size_t>(L.np);
  T* hist = a.p.hist;
  const int s_new = a.k & 3;
  const int s1 = (a.k + 3) & 3, s2 = (a.k + 2) & 3, s3 = (a.k + 1) & 3, s4 = s_new;
  unsigned int nclamp = 0, nabs = 0, nglob = 0;

  if constexpr (MODE == kTrialLater)
    trial_later_particles<T, O, nch>(L, a, tile, ts, I0, J0, ox, oy, nx, ny, tiled, owner, nglob);
  for (int e = threadIdx.x; MODE != kTrialLater && e < ts.tx * ts.ty; e += kBlock) {
    const int I = I0 + e % ts.tx, J = J0 + e / ts.tx;
    const size_t p = static_cast<size_t>(J) * L.nX + I;
    // every load of the particle is issued before any decision on it
    const T w = a.p.w[p];
    T xi = a.p.xi_x[p], eta = a.p.xi_y[p];
    T ux = a.p.ux[p], uy = a.p.uy[p], psi = a.p.psi[p];
    const int ci0 = I >> ts.lpx, cj0 = J >> ts.lpy;
    const T fx0 = (T(2 * (I & (L.ppc_x - 1)) + 1)) / T(2 * L.ppc_x);
    const T fy0 = (T(2 * (J & (L.ppc_y - 1)) + 1)) / T(2 * L.ppc_y);
    bool alive = w != T(0);

    if (MODE != kDepositOnly) {
      // the history part P_k of the step (written by the previous real push)
      // and, for the real push, f_{k-1}, f_{k-2}, f_{k-3} (which form P_{k+1}
      // with f_k); a taped push reads every slot for the tape
      T pk[5];
      T h[4][5];
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        pk[c] = a.p.pab[c * np + p];
        if constexpr (MODE == kPushReal || TAPE) {
          h[0][c] = hist[(s1 * 5 + c) * np + p];
          h[1][c] = hist[(s2 * 5 + c) * np + p];
          h[2][c] = hist[(s3 * 5 + c) * np + p];
        }
        if constexpr (TAPE) h[3][c] = hist[(s4 * 5 + c) * np + p];
      }
      if constexpr (MODE == kPushTrial && TAPE) {
        // the state the reverse pass of this slice starts from
        T* t = a.tape;
        t[p] = xi;
        t[np + p] = eta;
        t[2 * np + p] = ux;
        t[3 * np + p] = uy;
        t[4 * np + p] = psi;
        t[5 * np + p] = w;
        T* th = t + 6 * np;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          th[(s1 * 5 + c) * np + p] = h[0][c];
          th[(s2 * 5 + c) * np + p] = h[1][c];
          th[(s3 * 5 + c) * np + p] = h[2][c];
          th[(s4 * 5 + c) * np + p] = h[3][c];
        }
      }
      T e1, e2, ez, bx, by, bz;
      if constexpr (O == 1) {
        int ci, cj;
        const T fx = shape::locate<1>(ci0, fx0 + xi, nx, ci);
        const T fy = shape::locate<1>(cj0, fy0 + eta, ny, cj);
        const T w00 = (T(1) - fx) * (T(1) - fy), w10 = fx * (T(1) - fy);
        const T w01 = (T(1) - fx) * fy, w11 = fx * fy;
        e1 = gather(a.f.exmby, ci, cj, w00, w10, w01, w11, nx, ny);
        e2 = gather(a.f.eypbx, ci, cj, w00, w10, w01, w11, nx, ny);
        ez = gather(a.f.ez, ci, cj, w00, w10, w01, w11, nx, ny);
        bx = gather(a.f.bx, ci, cj, w00, w10, w01, w11, nx, ny);
        by = gather(a.f.by, ci, cj, w00, w10, w01, w11, nx, ny);
        bz = gather(a.f.bz, ci, cj, w00, w10, w01, w11, nx, ny);
      } else {
        int bi, bj;
        const T dx = shape::locate<O>(ci0, fx0 + xi, nx, bi);
        const T dy = shape::locate<O>(cj0, fy0 + eta, ny, bj);
        T wx[O + 1], wy[O + 1];
        int ix[O + 1], iy[O + 1];
        bool okx[O + 1], oky[O + 1];
        shape::weights<O>(dx, wx);
        shape::weights<O>(dy, wy);
        shape::axis_nodes<O>(bi, nx, ix, okx);
        shape::axis_nodes<O>(bj, ny, iy, oky);
#pragma unroll
        for (int q = 0; q <= O; ++q) {
          wx[q] = okx[q] ? wx[q] : T(0);
          wy[q] = oky[q] ? wy[q] : T(0);
        }
        e1 = shape::interp<O>(a.f.exmby, ix, iy, wx, wy, nx);
        e2 = shape::interp<O>(a.f.eypbx, ix, iy, wx, wy, nx);
        ez = shape::interp<O>(a.f.ez, ix, iy, wx, wy, nx);
        bx = shape::interp<O>(a.f.bx, ix, iy, wx, wy, nx);
        by = shape::interp<O>(a.f.by, ix, iy, wx, wy, nx);
        bz = shape::interp<O>(a.f.bz, ix, iy, wx, wy, nx);
      }
      // right-hand side of the pusher equations for an electron (q = -1)
      const T draw = T(1) + psi;
      const T d = draw < floor_d ? floor_d : draw;
      if (MODE == kPushReal && alive && draw < floor_d) ++nclamp;
      const T id = T(1) / d;
      const T gam = (T(1) + ux * ux + uy * uy + d * d) * T(0.5) * id;
      T f[5];
      f[0] = -ux * id * inv_hx;
      f[1] = -uy * id * inv_hy;
      if constexpr (MODE == kPushTrial) {   // the Bx/By kick is added below
        f[2] = gam * id * e1 + bz * uy * id;
        f[3] = gam * id * e2 - bz * ux * id;
      } else {
        f[2] = gam * id * e1 + by + bz * uy * id;
        f[3] = gam * id * e2 - bx - bz * ux * id;
      }
      f[4] = (ux * e1 + uy * e2) * id - ez;
      T y[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) y[c] = pk[c] - dz * (b0 * f[c]);
      if constexpr (MODE == kPushTrial) {
        const T cx = y[2], cy = y[3];
        const T kick = dz * b0;
        y[2] = cx - kick * by;
        y[3] = cy + kick * bx;
        if (a.rec) {   // what the later iterations of this slice start from
          const bool in_box = inside(ci0, fx0 + y[0], nx) && inside(cj0, fy0 + y[1], ny);
          const T dn = T(1) + y[4];
          const T idn = T(1) / (dn < floor_d ? floor_d : dn);
          T* r = a.rec;
          r[p] = y[0];
          r[np + p] = y[1];
          r[2 * np + p] = cx;
          r[3 * np + p] = cy;
          r[4 * np + p] = alive && in_box ? -w * idn : T(0);
          r[5 * np + p] = y[4];
        }
      }
      if (!alive) continue;
      if (!inside(ci0, fx0 + y[0], nx) || !inside(cj0, fy0 + y[1], ny)) {
        ++nabs;
        if (MODE == kPushReal) a.p.w[p] = T(0);
        continue;
      }
      xi = y[0];
      eta = y[1];
      ux = y[2];
      uy = y[3];
      psi = y[4];
      if constexpr (MODE == kPushReal) {
        a.p.xi_x[p] = xi;
        a.p.xi_y[p] = eta;
        a.p.ux[p] = ux;
        a.p.uy[p] = uy;
        a.p.psi[p] = psi;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          hist[(s_new * 5 + c) * np + p] = f[c];
          a.p.pab[c * np + p] = ab5_history(y[c], f[c], h[0][c], h[1][c], h[2][c], dz);
        }
      }
    } else if (!alive) {
      continue;
    }

    // deposit at the (new) position: rho - Jz = q w exactly, J = q w u / D
    const T draw = T(1) + psi;
    const bool clamped = draw < floor_d;
    const T d = clamped ? floor_d : draw;
    const T id = T(1) / d;
    const T omd = clamped ? T(1) - d : -psi;     // 1 - D
    double v[4];
    if (MODE == kPushTrial) {
      v[0] = static_cast<double>(-w * ux * id);
      v[1] = static_cast<double>(-w * uy * id);
    } else {
      const T u2 = ux * ux + uy * uy;
      const T uz = (u2 + omd * (T(1) + d)) * T(0.5) * id;
      v[0] = static_cast<double>(-w);
      v[1] = static_cast<double>(-w * ux * id);
      v[2] = static_cast<double>(-w * uy * id);
      v[3] = static_cast<double>(-w * uz * id);
    }
    deposit_particle<T, O, nch>(a.dep, tile, ts, ox, oy, nx, ny, tiled, owner, ci0, cj0, fx0, fy0,
                                xi, eta, v, nglob);
  }

  if (tiled) {
    __syncthreads();
    if (owner)
      flush_tile_owned<nch>(a.dep.ch, a.dep.sh, tile, ts, ox, oy, nx, ny);
    else
      flush_tile<nch>(a.dep.ch, tile, ts, ox, oy, nx, ny);
  }
  // counters (none of them is kept for a trial push)
  if constexpr (trial) return;
  const unsigned long long tc = block_sum(nclamp, red);
  const unsigned long long ta = block_sum(nabs, red);
  const unsigned long long tg = block_sum(nglob, red);
  if (threadIdx.x == 0) {
    if (tc) atomicAdd(&ctr->n_clamped, tc);
    if (MODE == kPushReal && ta) atomicAdd(&ctr->n_absorbed, ta);
    if (!trial && tg) atomicAdd(&ctr->n_dep_global, tg);
  }
}

// Sources of the explicit Bx/By solver for the particles of lattice tile
// (tbx, tby) at their slice-k state, in the final psi, Ez, Bz of slice k
// (shape order O >= 1).  Along the pusher's orbits (dx_p/dzeta = -u/D)
//   d_zeta J_perp = sum q w [ S d(u/D)/dzeta - (u/D) (grad_p S . u/D) ],
// whose B_perp part is -chi By (x) and +chi Bx (y) with chi = sum w S / D;
// the rest (DJx, DJy) and chi are deposited into dep.ch[0..2] = chi, DJx,
// DJy (FP64).  du/dzeta without B_perp: a_x = gamma/D (Ex-By) + Bz u_y/D,
// a_y = gamma/D (Ey+Bx) - Bz u_x/D; dPsi/dzeta = u.(E-vxB)_perp/D - Ez, and
// a floored D does not change.
template <typename T, int O>
__device__ __forceinline__ void explicit_tile(const Geom& g, const Lattice& L,
                                              const PushArgs<T>& a, int tbx, int tby,
                                              double* tile) {
  constexpr int nch = 3;
  const TileShape ts = tile_shape(L, a.tile_rows, a.tile_halo);
  const int ntile = ts.nw * ts.nh;
  const bool tiled = a.tiled != 0;
  if (tiled) {
    __syncthreads();
    for (int e = threadIdx.x; e < nch * ntile; e += kBlock) tile[e] = 0.0;
    __syncthreads();
  }
  const int I0 = tbx * ts.tx, J0 = tby * ts.ty;
  const int ox = (I0 >> ts.lpx) - ts.halo, oy = (J0 >> ts.lpy) - ts.halo;
  const int nx = g.nx, ny = g.ny;
  const double ihx = 1.0 / a.hx, ihy = 1.0 / a.hy;
  const T floor_d = static_cast<T>(a.psi_floor);

  for (int e = threadIdx.x; e < ts.tx * ts.ty; e += kBlock) {
    const int I = I0 + e % ts.tx, J = J0 + e / ts.tx;
    const size_t p = static_cast<size_t>(J) * L.nX + I;
    const T w = a.p.w[p];
    const T xi = a.p.xi_x[p], eta = a.p.xi_y[p];
    const T ux = a.p.ux[p], uy = a.p.uy[p], psi = a.p.psi[p];
    const int ci0 = I >> ts.lpx, cj0 = J >> ts.lpy;
    const T fx0 = (T(2 * (I & (L.ppc_x - 1)) + 1)) / T(2 * L.ppc_x);
    const T fy0 = (T(2 * (J & (L.ppc_y - 1)) + 1)) / T(2 * L.ppc_y);
    int bi, bj;
    const T dx = shape::locate<O>(ci0, fx0 + xi, nx, bi);
    const T dy = shape::locate<O>(cj0, fy0 + eta, ny, bj);
    T wx[O + 1], wy[O + 1];
    int ix[O + 1], iy[O + 1];
    bool okx[O + 1], oky[O + 1];
    shape::weights<O>(dx, wx);
    shape::weights<O>(dy, wy);
    shape::axis_nodes<O>(bi, nx, ix, okx);
    shape::axis_nodes<O>(bj, ny, iy, oky);
#pragma unroll
    for (int q = 0; q <= O; ++q) {
      wx[q] = okx[q] ? wx[q] : T(0);
      wy[q] = oky[q] ? wy[q] : T(0);
    }
    const T e1 = shape::interp<O>(a.f.exmby, ix, iy, wx, wy, nx);
    const T e2 = shape::interp<O>(a.f.eypbx, ix, iy, wx, wy, nx);
    const T ez = shape::interp<O>(a.f.ez, ix, iy, wx, wy, nx);
    const T bz = shape::interp<O>(a.f.bz, ix, iy, wx, wy, nx);
    if (w == T(0)) continue;
    const T draw = T(1) + psi;
    const bool clamped = draw < floor_d;
    const T d = clamped ? floor_d : draw;
    const T id = T(1) / d;
    const T gam = (T(1) + ux * ux + uy * uy + d * d) * T(0.5) * id;
    const T ax = gam * id * e1 + bz * uy * id;
    const T ay = gam * id * e2 - bz * ux * id;
    const T apsi = clamped ? T(0) : (ux * e1 + uy * e2) * id - ez;
    const T qn = -w;
    const double cx = static_cast<double>(qn * (ax * id - ux * apsi * id * id));
    const double cy = static_cast<double>(qn * (ay * id - uy * apsi * id * id));
    const double vx = static_cast<double>(ux * id), vy = static_cast<double>(uy * id);
    const double qd = static_cast<double>(qn);
    const double chi_p = static_cast<double>(w * id);
    double sx[O + 1], sy[O + 1], gx[O + 1], gy[O + 1];
    shape::weights<O>(static_cast<double>(dx), sx);
    shape::weights<O>(static_cast<double>(dy), sy);
    shape::weight_slopes<O>(static_cast<double>(dx), gx);
    shape::weight_slopes<O>(static_cast<double>(dy), gy);
    const int li = bi - ox, lj = bj - oy;
    const bool in_tile = tiled && li >= 0 && li + O < ts.nw && lj >= 0 && lj + O < ts.nh;
#pragma unroll
    for (int qb = 0; qb <= O; ++qb) {
      const int gj = bj + qb;
#pragma unroll
      for (int qa = 0; qa <= O; ++qa) {
        const int gi = bi + qa;
        const double sw = sx[qa] * sy[qb];
        const double vg = vx * (gx[qa] * sy[qb] * ihx) + vy * (sx[qa] * gy[qb] * ihy);
        const double v0 = chi_p * sw;
        // (u/D) dS/dzeta with dS/dzeta = -(grad_p S . u/D) = -vg
        const double v1 = cx * sw - qd * vx * vg;
        const double v2 = cy * sw - qd * vy * vg;
        if (in_tile) {
          double* t = tile + (lj + qb) * ts.nw + (li + qa);
          lds_add(t, v0);
          lds_add(t + ntile, v1);
          lds_add(t + 2 * ntile, v2);
        } else if (gi >= 1 && gi < nx && gj >= 1 && gj < ny) {
          const size_t o = static_cast<size_t>(gj) * nx + gi;
          global_add(a.dep.ch[0] + o, v0);
          global_add(a.dep.ch[1] + o, v1);
          global_add(a.dep.ch[2] + o, v2);
        }
      }
    }
  }

  if (tiled) {
    __syncthreads();
    flush_tile<nch>(a.dep.ch, tile, ts, ox, oy, nx, ny);
  }
}

}  // namespace push_detail
}  // namespace qsp
