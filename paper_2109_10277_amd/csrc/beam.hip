// Macro-particle beams (HiPACE++, arXiv:2109.10277, Sec. III.A): the beam is
// sorted by slice once per box, and inside the slice loop the particles of
// slice k deposit their charge and longitudinal current (zeroth order in
// zeta, transverse shape of order 0-3) before the field solves, then take one time step
// (second-order drift-kick-drift with a Boris kick) in the fields of slice k
// once those are final.  The slice sort is a stable counting sort.
#include "common.hpp"
#include "kernels.hpp"
#include "shape.hpp"

namespace qsp {

namespace {

dim3 grid_of(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 65535 * 16) b = 65535 * 16;
  return dim3(static_cast<unsigned>(b));
}

// Stable counting sort by nearest slice.  The particles are cut into chunks
// of kSortChunk consecutive ones, one 64-lane workgroup each; keys are
// 0..nzeta (nzeta: outside the box), counted in LDS.
//   hist     per chunk, the count of each key          [nchunk][nkey]
//   colscan  per key, the exclusive prefix over chunks (in place) and the total
//   keyscan  exclusive prefix of the totals: off[k] = first particle of key k
//   scatter  each chunk again, in order, 64 particles a round: a particle's
//            place is off[k] + (earlier chunks' k) + (earlier rounds' k) + (k
//            among the lower lanes of its round), found with one ballot per
//            key bit; all seven components move to it.
constexpr int kSortLanes = 64;
constexpr int kSortRounds = 64;
constexpr int kSortChunk = kSortLanes * kSortRounds;

__device__ inline int slice_key(float z, double zeta_hi, double dzeta, int nzeta) {
  const double s = rint((zeta_hi - static_cast<double>(z)) / dzeta);   // nearest slice
  return s >= 0.0 && s < static_cast<double>(nzeta) ? static_cast<int>(s) : nzeta;
}

__global__ void __launch_bounds__(kSortLanes)
k_sort_hist(const float* __restrict__ soa, int64_t n, double zeta_hi, double dzeta, int nzeta,
            int* __restrict__ hist) {
  extern __shared__ int cnt[];
  const int nkey = nzeta + 1;
  const int lane = static_cast<int>(threadIdx.x);
  for (int k = lane; k < nkey; k += kSortLanes) cnt[k] = 0;
  __syncthreads();
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kSortChunk;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = c0 + r * kSortLanes + lane;
    if (i < n) atomicAdd(&cnt[slice_key(soa[2 * n + i], zeta_hi, dzeta, nzeta)], 1);
  }
  __syncthreads();
  int* h = hist + static_cast<int64_t>(blockIdx.x) * nkey;
  for (int k = lane; k < nkey; k += kSortLanes) h[k] = cnt[k];
}

// one thread per key: column prefix over the chunks, in place, and the total
__global__ void k_sort_colscan(int* __restrict__ hist, int nchunk, int nkey, int* __restrict__ total) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nkey) return;
  constexpr int U = 8;
  int run = 0;
  int c = 0;
  for (; c + U <= nchunk; c += U) {
    int v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = hist[static_cast<int64_t>(c + u) * nkey + k];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      hist[static_cast<int64_t>(c + u) * nkey + k] = run;
      run += v[u];
    }
  }
  for (; c < nchunk; ++c) {
    const int v = hist[static_cast<int64_t>(c) * nkey + k];
    hist[static_cast<int64_t>(c) * nkey + k] = run;
    run += v;
  }
  total[k] = run;
}

// one workgroup: off[k] = sum of total[k'] for k' < k, k = 0..nkey
__global__ void __launch_bounds__(kBlock)
k_sort_keyscan(const int* __restrict__ total, int nkey, int64_t* __restrict__ off) {
  __shared__ int64_t part[kBlock];
  const int t = static_cast<int>(threadIdx.x);
  const int per = (nkey + kBlock - 1) / kBlock;
  const int k0 = t * per, k1 = min(nkey, k0 + per);
  int64_t s = 0;
  for (int k = k0; k < k1; ++k) s += total[k];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int u = 0; u < kBlock; ++u) {
      const int64_t v = part[u];
      part[u] = run;
      run += v;
    }
    off[nkey] = run;
  }
  __syncthreads();
  int64_t run = part[t];
  for (int k = k0; k < k1; ++k) {
    off[k] = run;
    run += total[k];
  }
}

__global__ void __launch_bounds__(kSortLanes)
k_sort_scatter(const float* __restrict__ in, int64_t n, double zeta_hi, double dzeta, int nzeta,
               int kbits, const int* __restrict__ hist, const int64_t* __restrict__ off,
               float* __restrict__ out) {
  extern __shared__ int pos[];
  const int nkey = nzeta + 1;
  const int lane = static_cast<int>(threadIdx.x);
  const int* h = hist + static_cast<int64_t>(blockIdx.x) * nkey;
  for (int k = lane; k < nkey; k += kSortLanes) pos[k] = static_cast<int>(off[k]) + h[k];
  __syncthreads();
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kSortChunk;
  const uint64_t below = (uint64_t{1} << lane) - 1;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = c0 + r * kSortLanes + lane;
    const bool valid = i < n;
    const int key = valid ? slice_key(in[2 * n + i], zeta_hi, dzeta, nzeta) : 0;
    // lanes of the round with the same key
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < kbits; ++b) {
      const bool bit = (key >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    // every peer reads the key's position before the lowest peer advances it
    // (one wave: its LDS operations complete in order)
    const int base = valid ? pos[key] : 0;
    __builtin_amdgcn_wave_barrier();
    if (valid && (peers & below) == 0) pos[key] = base + __popcll(peers);
    if (valid) {
      const int64_t d = base + __popcll(peers & below);
#pragma unroll
      for (int c = 0; c < 7; ++c) out[c * n + d] = in[c * n + i];
    }
    __builtin_amdgcn_wave_barrier();
  }
}

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

}  // namespace

// rho = q w / (hx hy dzeta), Jz = rho u_z / gamma, rho - Jz written as
// rho (1 + u_perp^2) / (gamma (gamma + u_z)) so that it does not cancel
// The particles of slice k are off[k] .. off[k+1]-1 of the sorted beam; the
// range is read on the device (a captured box stays valid when the beam is
// sorted again between boxes) and covered by a grid-stride loop.
template <int O>
__global__ void k_beam_deposit(Geom g, const float* __restrict__ soa, int64_t n,
                               const int64_t* __restrict__ off, int k, double dzeta,
                               double* rho_mjz, double* jz, double* rho) {
  const int64_t start = off[k], count = off[k + 1] - start;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < count;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t p = start + t;
    const double x = soa[p], y = soa[n + p];
    const double ux = soa[3 * n + p], uy = soa[4 * n + p], uz = soa[5 * n + p], w = soa[6 * n + p];
    double sx, sy;
    if (!node_coord(x, g.x_lo, g.hx, g.nx, sx) || !node_coord(y, g.y_lo, g.hy, g.ny, sy)) continue;
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

template <typename T, int O>
__global__ void k_beam_push(Geom g, float* soa, int64_t n, const int64_t* __restrict__ off, int k,
                            SliceFields<T> f, double dt) {
  const int64_t start = off[k], count = off[k + 1] - start;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < count;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x)
    beam_push_one<T, O>(g, soa, n, start + t, f, dt);
}

// ------------------------------------------------------------------ host side
int beam_sort_chunks(int64_t n) { return static_cast<int>((n + kSortChunk - 1) / kSortChunk); }

void beam_sort(const float* in, float* out, int64_t n, double zeta_hi, double dzeta, int nzeta,
               BeamScratch& s, std::vector<int64_t>& offsets, hipStream_t st) {
  const int nkey = nzeta + 1;
  if (nkey > kMaxBeamKeys) throw std::invalid_argument("particle beams need nzeta < 16384");
  const int nchunk = beam_sort_chunks(n);
  if (nchunk > s.nchunk) throw std::runtime_error("beam sort scratch too small");
  int kbits = 1;
  while ((1 << kbits) < nkey) ++kbits;
  const size_t lds = static_cast<size_t>(nkey) * sizeof(int);
  hipLaunchKernelGGL(k_sort_hist, dim3(nchunk), dim3(kSortLanes), lds, st, in, n, zeta_hi, dzeta,
                     nzeta, s.hist);
  QSP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sort_colscan, dim3((nkey + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                     s.hist, nchunk, nkey, s.total);
  QSP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sort_keyscan, dim3(1), dim3(kBlock), 0, st, s.total, nkey, s.off);
  QSP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sort_scatter, dim3(nchunk), dim3(kSortLanes), lds, st, in, n, zeta_hi, dzeta,
                     nzeta, kbits, s.hist, s.off, out);
  QSP_LAUNCH_CHECK();
  offsets.assign(nzeta + 2, 0);
  QSP_HIP(hipMemcpyAsync(offsets.data(), s.off, (nzeta + 2) * sizeof(int64_t),
                         hipMemcpyDeviceToHost, st));
  QSP_HIP(hipStreamSynchronize(st));
}

void launch_beam_deposit(const Geom& g, const float* soa, int64_t n, const int64_t* off, int k,
                         int64_t grid_count, double dzeta, double* rho_mjz, double* jz,
                         double* rho, hipStream_t st) {
  if (k < 0 || grid_count < 1) throw std::invalid_argument("beam deposit: bad slice or grid");
  with_order(g.order, [&](auto order) {
    hipLaunchKernelGGL((k_beam_deposit<decltype(order)::value>), grid_of(grid_count), dim3(kBlock),
                       0, st, g, soa, n, off, k, dzeta, rho_mjz, jz, rho);
  });
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_beam_push(const Geom& g, float* soa, int64_t n, const int64_t* off, int k,
                      int64_t grid_count, const SliceFields<T>& f, double dt, hipStream_t st) {
  if (k < 0 || grid_count < 1) throw std::invalid_argument("beam push: bad slice or grid");
  with_order(g.order, [&](auto order) {
    hipLaunchKernelGGL((k_beam_push<T, decltype(order)::value>), grid_of(grid_count), dim3(kBlock),
                       0, st, g, soa, n, off, k, f, dt);
  });
  QSP_LAUNCH_CHECK();
}

template void launch_beam_push<float>(const Geom&, float*, int64_t, const int64_t*, int, int64_t,
                                      const SliceFields<float>&, double, hipStream_t);
template void launch_beam_push<double>(const Geom&, float*, int64_t, const int64_t*, int, int64_t,
                                       const SliceFields<double>&, double, hipStream_t);

}  // namespace qsp
