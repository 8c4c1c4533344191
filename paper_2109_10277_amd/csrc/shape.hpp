// Transverse particle shapes of orders 0-3 (HiPACE++, arXiv:2109.10277
// Sec. III.B: deposition is zeroth order in zeta and of order 0 to 3
// transversely).  Order p is the centred cardinal B-spline of degree p, used
// as a tensor product in x and y for the deposit and, transposed, for the
// field gather:
//   order 0  nearest node                    1 node
//   order 1  linear (CIC)                    2 nodes
//   order 2  quadratic, centred on the nearest node   3 nodes
//   order 3  cubic, around the particle's cell        4 nodes
// A position is given as node coordinate s = c0 + t, with c0 an integer and
// t the offset in cells, so that the fraction inside the stencil is formed
// without cancellation.  Stencil nodes outside 0..n are returned as they
// are: callers drop them in a deposit and read them as zero in a gather.
// Order 1 keeps its cell inside 0..n-1 (s = n uses cell n-1 with weight 1 on
// node n), which changes no weight.
#pragma once

#include <hip/hip_runtime.h>

#include <stdexcept>
#include <type_traits>

namespace qsp {
namespace shape {

// lowest stencil node b and fraction d of a particle at s = c0 + t:
//   order 1, 3: d = s - floor(s) in [0, 1), b = floor(s) - (order == 3)
//   order 0, 2: d = s - round(s) in [-1/2, 1/2) (halves round up),
//               b = round(s) - (order == 2)
template <int O, typename T>
__host__ __device__ __forceinline__ T locate(int c0, T t, int n, int& b) {
  const T fl = floor(t);
  T d = t - fl;                       // exact
  int c = c0 + static_cast<int>(fl);
  if constexpr (O == 1) {
    if (c >= n) {
      c = n - 1;
      d = T(1);
    }
    if (c < 0) {
      c = 0;
      d = T(0);
    }
    b = c;
  } else if constexpr (O == 3) {
    b = c - 1;
  } else {
    if (d >= T(0.5)) {
      d -= T(1);
      ++c;
    }
    b = c - (O == 2 ? 1 : 0);
  }
  return d;
}

// B-spline weights of the O+1 stencil nodes for fraction d
template <int O, typename R>
__host__ __device__ __forceinline__ void weights(R d, R (&w)[O + 1]) {
  if constexpr (O == 0) {
    w[0] = R(1);
  } else if constexpr (O == 1) {
    w[0] = R(1) - d;
    w[1] = d;
  } else if constexpr (O == 2) {
    const R a = R(0.5) - d, c = R(0.5) + d;
    w[0] = R(0.5) * a * a;
    w[1] = R(0.75) - d * d;
    w[2] = R(0.5) * c * c;
  } else {
    const R e = R(1) - d, d2 = d * d, d3 = d2 * d;
    const R s6 = R(1) / R(6);
    w[0] = e * e * e * s6;
    w[1] = (R(4) - R(6) * d2 + R(3) * d3) * s6;
    w[2] = (R(1) + R(3) * d + R(3) * d2 - R(3) * d3) * s6;
    w[3] = d3 * s6;
  }
}

// derivatives of the weights with respect to the position (per cell)
template <int O, typename R>
__host__ __device__ __forceinline__ void weight_slopes(R d, R (&g)[O + 1]) {
  if constexpr (O == 0) {
    g[0] = R(0);
  } else if constexpr (O == 1) {
    g[0] = R(-1);
    g[1] = R(1);
  } else if constexpr (O == 2) {
    g[0] = d - R(0.5);
    g[1] = R(-2) * d;
    g[2] = R(0.5) + d;
  } else {
    const R e = R(1) - d;
    g[0] = R(-0.5) * e * e;
    g[1] = (R(-2) + R(1.5) * d) * d;
    g[2] = R(0.5) + d - R(1.5) * d * d;
    g[3] = R(0.5) * d * d;
  }
}

// clamped node indices of a stencil axis (all loads stay in 0..n-1) and a
// mask of the nodes that are stored: 0 <= node < n (node n and beyond are
// Dirichlet or outside, node 0 is stored as zero)
template <int O>
__host__ __device__ __forceinline__ void axis_nodes(int b, int n, int (&idx)[O + 1], bool (&ok)[O + 1]) {
#pragma unroll
  for (int a = 0; a <= O; ++a) {
    const int v = b + a;
    ok[a] = v >= 0 && v < n;
    idx[a] = v < 0 ? 0 : (v >= n ? n - 1 : v);
  }
}

// sum_b wy[b] sum_a wx[a] F[j_b][i_a] over the stored nodes of the stencil
template <int O, typename T, typename R>
__device__ __forceinline__ R interp(const T* __restrict__ F, const int (&ix)[O + 1],
                                    const int (&iy)[O + 1], const R (&wx)[O + 1],
                                    const R (&wy)[O + 1], int nx) {
  R v = R(0);
#pragma unroll
  for (int b = 0; b <= O; ++b) {
    const T* row = F + static_cast<size_t>(iy[b]) * nx;
    R r = R(0);
#pragma unroll
    for (int a = 0; a <= O; ++a) r += wx[a] * static_cast<R>(row[ix[a]]);
    v += wy[b] * r;
  }
  return v;
}

}  // namespace shape

// calls f(std::integral_constant<int, order>{}) for a run-time shape order
template <typename F>
inline void with_order(int order, F&& f) {
  switch (order) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    default: throw std::invalid_argument("shape order must be 0, 1, 2 or 3");
  }
}

}  // namespace qsp
