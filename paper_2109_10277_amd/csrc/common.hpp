// Shared declarations of the libqsp runtime and its HIP kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace qsp {

// 256 threads = 4 wave64 wavefronts per workgroup everywhere.
constexpr int kBlock = 256;

// Largest number of output copies one slice can request (12 quantities as
// full plane, centre row and axis node).
constexpr int kMaxOut = 36;

// Fifth-order Adams-Bashforth weights (numerators over 720) for
// f_k, f_{k-1}, ..., f_{k-4}.
constexpr double kAB5[5] = {1901.0 / 720.0, -2774.0 / 720.0, 2616.0 / 720.0,
                            -1274.0 / 720.0, 251.0 / 720.0};

// History part of an Adams-Bashforth step from slice k: y_k - dz (b1 f_{k-1}
// + b2 f_{k-2} + b3 f_{k-3} + b4 f_{k-4}), so that y_{k+1} = P_k - dz b0 f_k.
// One function for every place that forms it (the real push, state import,
// checkpoint restore), so that they round alike.
template <typename T>
__host__ __device__ __forceinline__ T ab5_history(T y, T f1, T f2, T f3, T f4, T dz) {
  return y - dz * (T(kAB5[1]) * f1 + T(kAB5[2]) * f2 + T(kAB5[3]) * f3 + T(kAB5[4]) * f4);
}

struct DeviceError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

inline void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e != hipSuccess) {
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%s failed at %s:%d: %s", what, file, line,
                  hipGetErrorString(e));
    throw DeviceError(buf);
  }
}
#define QSP_HIP(call) ::qsp::hip_check((call), #call, __FILE__, __LINE__)
#define QSP_LAUNCH_CHECK() ::qsp::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

template <typename T>
struct Cplx {
  T re, im;
};

// ---------------------------------------------------------------------------
// Grid geometry shared by all kernels.  Node arrays are stored [ny][nx]
// (pitch nx): element (j, i) is node (i, j) for i, j in 0..n-1; node index 0
// carries the Dirichlet boundary (always 0 for fields) and node index n is
// implicit (0).  This makes each stored row the first half of the odd
// extension a type-I sine transform needs.
// ---------------------------------------------------------------------------
struct Geom {
  int nx, ny;            // cells = nodes per stored row/column
  int lx, ly;            // log2(nx), log2(ny)
  double x_lo, y_lo, hx, hy;
  int rr;                // rows per workgroup of the transform row passes
  int order;             // transverse particle shape order, 0..3
  // 1: the planes between the row and column passes of a solve are stored
  // in strips of 4 columns, element (j, i) at ((i / 4) ny + j) 4 + i % 4
  // (FP32 at 1024^2: the column pass reads and writes one contiguous
  // block per strip, the row passes 64-byte blocks of 4 rows x 4 columns);
  // 0: row-major
  int strip;
};

// Offset of element (j, i) of a strip-ordered intermediate plane.
__host__ __device__ inline size_t strip_at(int j, int i, int ny) {
  return (static_cast<size_t>(i >> 2) * ny + j) * 4 + (i & 3);
}

// Plasma lattice: (nx*ppc_x) x (ny*ppc_y) sites, particle p = I + J*nX.
struct Lattice {
  int nX, nY, ppc_x, ppc_y;
  int64_t np;
};

// Sine transforms of FP32 rows of 256-1024 points use the recurrence-free
// core (an FFT of the odd extension, twice the length); the others the
// half-length transform with a prefix sum for the odd outputs.
__host__ __device__ constexpr bool fast_core(int elem_size, int n) {
  return elem_size == 4 && n >= 256 && n <= 1024;
}

// Lanes that transform one row pair with the FP32 core: two waves (128) at
// 1024 points, one wave (64) at 256 and 512 (two waves measured slower
// there: 512^2 column pass 10.3 against 8.3 us).
__host__ __device__ constexpr int core_lanes(int elem_size, int n) {
  return fast_core(elem_size, n) && n >= 1024 ? 128 : 64;
}

// Per-axis transform tables (device pointers): for the half-length
// transform tw[m] = e^{-2 pi i m / n} and pre[j] = sin(pi j / n); for the
// FP32 core with NL = core_lanes lanes per pair tw[k1 * NL + l] =
// e^{-2 pi i l k1 / 2n} (2n entries) and pre holds the complex table
// W_NL^{la c1} at [la * 9 + c1] (la < NL / 8, c1 < 8, entry 8 of a row 0).
template <typename T>
struct AxisTables {
  const Cplx<T>* tw;
  const T* pre;
  const double* lam;     // Laplacian eigenvalue of sine mode p, p = 0..n-1 (0 unused)
};

// Device-side scalars of the predictor-corrector and counters.
struct DevCounters {
  unsigned int pc_done;        // 1 once the current slice's P-C converged
  unsigned int pc_iters;       // iterations done for the current slice
  unsigned int nonfinite;      // sticky: non-finite residual or norm seen
  double pc_resid;             // last residual of the current slice
  double max_resid;            // largest final residual over slices
  unsigned long long n_clamped;
  unsigned long long n_absorbed;
  unsigned long long n_dep_global;
  unsigned long long pc_iterations;
  unsigned long long pc_not_converged;
  // slices whose launched iterations (a launch budget below the maximum)
  // ended before the predictor-corrector converged
  unsigned int budget_short;
  unsigned int reserved0;
};

}  // namespace qsp
