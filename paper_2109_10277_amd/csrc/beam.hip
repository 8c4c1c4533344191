// Macro-particle beams (HiPACE++, arXiv:2109.10277, Sec. III.A): the beam is
// sorted by slice once per box, and inside the slice loop the particles of
// slice k deposit their charge and longitudinal current (zeroth order in
// zeta, transverse shape of order 0-3) before the field solves, then take one time step
// (second-order drift-kick-drift with a Boris kick) in the fields of slice k
// once those are final.  The slice sort is a stable counting sort.
#include "common.hpp"
#include "kernels.hpp"
#include "shape.hpp"
#include "beam_body.hpp"

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

}  // namespace

// rho = q w / (hx hy dzeta), Jz = rho u_z / gamma, rho - Jz written as
// rho (1 + u_perp^2) / (gamma (gamma + u_z)) so that it does not cancel
template <int O>
__global__ void k_beam_deposit(Geom g, const float* __restrict__ soa, int64_t n,
                               const int64_t* __restrict__ off, int k, double dzeta,
                               double* rho_mjz, double* jz, double* rho) {
  beam_detail::beam_deposit_range<O>(g, soa, n, off, k, dzeta, rho_mjz, jz, rho,
                                     blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x,
                                     static_cast<int64_t>(gridDim.x) * blockDim.x);
}

template <typename T, int O>
__global__ void k_beam_push(Geom g, float* soa, int64_t n, const int64_t* __restrict__ off, int k,
                            SliceFields<T> f, double dt) {
  beam_detail::beam_push_range<T, O>(g, soa, n, off, k, f, dt,
                                     blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x,
                                     static_cast<int64_t>(gridDim.x) * blockDim.x);
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
