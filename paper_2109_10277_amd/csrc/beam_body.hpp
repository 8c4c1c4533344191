// Device bodies of the macro-particle beam kernels (HiPACE++,
// arXiv:2109.10277, Sec. III.A-B): deposit of rho - Jz, Jz (and rho) of one
// beam particle with the transverse shape of order O, zeroth order in zeta,
// and its time step (second-order drift-kick-drift with a Boris kick) in
// the fields of its slice.  Used by the beam kernels and by the real plasma
// push, whose launch also carries the beam work of its slice.
#pragma once

#include "common.hpp"
#include "kernels.hpp"
#include "shape.hpp"

namespace qsp {
namespace beam_detail {

// node coordinate of an absolute position; false outside [lo, lo + n h]
__device__ inline bool node_coord(double x, double lo, double h, int n, double& s) {
  s = (x - lo) / h;
  return s >= 0.0 && s <= static_cast<double>(n);
}

__device__ inline void add_node(double* p, int i, int j, int nx, int ny, double v) {
  if (i >= 1 && i < nx && j >= 1 && j < ny) unsafeAtomicAdd(p + static_cast<size_t>(j) * nx + i, v);
}

// shape weights of one axis, zero on the nodes that are not stored
template <int O>
__device__ inline void axis(double s, int n, int (&idx)[O + 1], double (&w)[O + 1]) {
  int b;
  const double d = shape::locate<O>(0, s, n, b);
  bool ok[O + 1];
  shape::weights<O>(d, w);
  shape::axis_nodes<O>(b, n, idx, ok);
#pragma unroll
  for (int a = 0; a <= O; ++a) w[a] = ok[a] ? w[a] : 0.0;
}

// Deposit of beam particle p: rho = q w / (hx hy dzeta), Jz = rho u_z /
// gamma, rho - Jz written as rho (1 + u_perp^2) / (gamma (gamma + u_z)) so
// that it does not cancel (any of the three planes may be null).
template <int O>
__device__ __forceinline__ void beam_deposit_one(const Geom& g, const float* __restrict__ soa,
                                                 int64_t n, int64_t p, double dzeta,
                                                 double* rho_mjz, double* jz, double* rho) {
  const double x = soa[p], y = soa[n + p];
  const double ux = soa[3 * n + p], uy = soa[4 * n + p], uz = soa[5 * n + p], w = soa[6 * n + p];
  double sx, sy;
  if (!node_coord(x, g.x_lo, g.hx, g.nx, sx) || !node_coord(y, g.y_lo, g.hy, g.ny, sy)) return;
  int bi, bj;
  double wx[O + 1], wy[O + 1];
  shape::weights<O>(shape::locate<O>(0, sx, g.nx, bi), wx);
  shape::weights<O>(shape::locate<O>(0, sy, g.ny, bj), wy);
  const double gam = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
  const double r = -w / (g.hx * g.hy * dzeta);
  const double v[3] = {r * (1.0 + ux * ux + uy * uy) / (gam * (gam + uz)), r * uz / gam, r};
  double* ch[3] = {rho_mjz, jz, rho};
  for (int c = 0; c < 3; ++c) {
    if (!ch[c]) continue;
#pragma unroll
    for (int qb = 0; qb <= O; ++qb)
#pragma unroll
      for (int qa = 0; qa <= O; ++qa)
        add_node(ch[c], bi + qa, bj + qb, g.nx, g.ny, v[c] * (wx[qa] * wy[qb]));
  }
}

// one time step of the particles of a slice in that slice's fields
template <typename T, int O>
__device__ __forceinline__ void beam_push_one(const Geom& g, float* soa, int64_t n, int64_t p,
                                              const SliceFields<T>& f, double dt) {
  double u[3] = {soa[3 * n + p], soa[4 * n + p], soa[5 * n + p]};
  const double g0 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const double xh = soa[p] + 0.5 * dt * u[0] / g0;
  const double yh = soa[n + p] + 0.5 * dt * u[1] / g0;
  const double zh = soa[2 * n + p] + 0.5 * dt * (u[2] / g0 - 1.0);
  double E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
  double sx, sy;
  if (node_coord(xh, g.x_lo, g.hx, g.nx, sx) && node_coord(yh, g.y_lo, g.hy, g.ny, sy)) {
    int ix[O + 1], iy[O + 1];
    double wx[O + 1], wy[O + 1];
    axis<O>(sx, g.nx, ix, wx);
    axis<O>(sy, g.ny, iy, wy);
    const double e1 = shape::interp<O>(f.exmby, ix, iy, wx, wy, g.nx);
    const double e2 = shape::interp<O>(f.eypbx, ix, iy, wx, wy, g.nx);
    B[0] = shape::interp<O>(f.bx, ix, iy, wx, wy, g.nx);
    B[1] = shape::interp<O>(f.by, ix, iy, wx, wy, g.nx);
    B[2] = shape::interp<O>(f.bz, ix, iy, wx, wy, g.nx);
    E[0] = e1 + B[1];
    E[1] = e2 - B[0];
    E[2] = shape::interp<O>(f.ez, ix, iy, wx, wy, g.nx);
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

// The particles of slice k are off[k] .. off[k+1]-1 of the sorted beam; the
// range is read on the device (a captured box stays valid when the beam is
// sorted again between boxes).  Thread t0 of a grid of `stride` threads
// takes every stride-th particle of the range.
template <int O>
__device__ __forceinline__ void beam_deposit_range(const Geom& g, const float* __restrict__ soa,
                                                   int64_t n, const int64_t* __restrict__ off,
                                                   int k, double dzeta, double* rho_mjz,
                                                   double* jz, double* rho, int64_t t0,
                                                   int64_t stride) {
  const int64_t start = off[k], count = off[k + 1] - start;
  for (int64_t t = t0; t < count; t += stride)
    beam_deposit_one<O>(g, soa, n, start + t, dzeta, rho_mjz, jz, rho);
}

template <typename T, int O>
__device__ __forceinline__ void beam_push_range(const Geom& g, float* soa, int64_t n,
                                                const int64_t* __restrict__ off, int k,
                                                const SliceFields<T>& f, double dt, int64_t t0,
                                                int64_t stride) {
  const int64_t start = off[k], count = off[k + 1] - start;
  for (int64_t t = t0; t < count; t += stride) beam_push_one<T, O>(g, soa, n, start + t, f, dt);
}

}  // namespace beam_detail
}  // namespace qsp
