// Batched 2D Dirichlet Poisson / Helmholtz solves with type-I sine transforms
// (fast Poisson solver of HiPACE++, arXiv:2109.10277 Sec. III.B), written for
// gfx950: every 1D transform runs inside LDS, two real rows packed into one
// complex FFT (Stockham, radix 8 with a radix-4/2 tail, one wavefront per
// group of row pairs), with a pre-twiddle that reduces the DST-I of length
// n-1 to a complex FFT of length n per row pair.
//
// Three passes per solve:
//   P1 (row pass)     source assembly (FP64 deposits -> T) fused with the
//                      forward DST along x, one workgroup per block of rows;
//   P2 (column pass)   forward DST along y, division by the eigenvalues of
//                      (lap_h - shift), inverse DST along y (plus an optional
//                      -d_y of the result), one workgroup per column strip;
//   P3 (row pass)     inverse DST along x with a fused epilogue (plain store,
//                      -d_x for Ex-By, or the predictor-corrector update with
//                      its FP64 residual reduction).
//
// Transform used (per row x_0..x_{n-1}, x_0 = x_n = 0):
//   S_p = sum_j x_j sin(pi j p / n).  With y_j = sin(pi j/n)(x_j + x_{n-j})
//   + (x_j - x_{n-j})/2 and Y = DFT_n(y): S_{2q} = -Im Y_q and
//   S_{2q+1} = S_{2q-1} + Re Y_q (S_1 = Re Y_0 / 2), i.e. odd outputs are a
//   prefix sum.  Two rows a, b are transformed together as DFT(y_a + i y_b).
//   Inverse: x = (2/n) S(S(x)); the 2D factor 4/(nx ny) is folded into the
//   eigenvalue division of P2.
#pragma once

#include <cstdlib>
#include <stdexcept>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "partials.hpp"

namespace qsp {
namespace dst_detail {

template <typename T>
__device__ inline Cplx<T> cmul(Cplx<T> a, Cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// LDS layout of a row pair.  One pad element per 128-byte bank row keeps the
// strided accesses of the FFT stages and of the odd-entry scan from piling
// onto the same banks.  Complex element m of a pair sits at cidx(m); real
// element i of row a at ridx(i), of row b at rlen(n) + ridx(i).
template <typename T>
struct Pad {
  static constexpr int cs = sizeof(T) == 4 ? 4 : 3;
  static constexpr int rs = sizeof(T) == 4 ? 5 : 4;
  __host__ __device__ static int cidx(int m) { return m + (m >> cs); }
  __host__ __device__ static int ridx(int i) { return i + (i >> rs); }
  __host__ __device__ static int rlen(int n) { return n + (n >> rs); }
  // T units per row pair (even, so complex views stay aligned)
  __host__ __device__ static int pitch(int n) {
    const int c = 2 * (n + (n >> cs)), r = 2 * rlen(n);
    return (c > r ? c : r) + 2;
  }
  __host__ __device__ static int rpos(int n, int pitch, int r, int i) {
    return (r >> 1) * pitch + (r & 1) * rlen(n) + ridx(i);
  }
};

// ---------------------------------------------------------------------------
// Wave-level transforms.  Each wavefront owns a group of P row pairs
// (P * n >= 512 complex points, P = max(1, 512 / n)) and transforms them in
// its own part of LDS: no workgroup barrier inside a transform.  LDS
// operations of one wavefront execute in order, so a wave-local exchange
// only needs the compiler kept from reordering across the sync point.
// ---------------------------------------------------------------------------
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ inline Cplx<T> cadd(Cplx<T> a, Cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ inline Cplx<T> csub(Cplx<T> a, Cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ inline Cplx<T> cmul_mi(Cplx<T> a) { return {a.im, -a.re}; }   // -i a

// in-place DFT of length 4 (forward)
template <typename T>
__device__ __forceinline__ void dft4(Cplx<T>& y0, Cplx<T>& y1, Cplx<T>& y2, Cplx<T>& y3) {
  const Cplx<T> c0 = cadd(y0, y2), c1 = csub(y0, y2), c2 = cadd(y1, y3);
  const Cplx<T> c3 = cmul_mi(csub(y1, y3));
  y0 = cadd(c0, c2);
  y2 = csub(c0, c2);
  y1 = cadd(c1, c3);
  y3 = csub(c1, c3);
}

// in-place DFT of length 8 (forward), natural order in and out
template <typename T>
__device__ __forceinline__ void dft8(Cplx<T>* v) {
  const T h = T(0.70710678118654752440);
  Cplx<T> a[4], b[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    a[m] = cadd(v[m], v[m + 4]);
    b[m] = csub(v[m], v[m + 4]);
  }
  // b_m *= e^{-2 pi i m / 8}
  b[1] = {h * (b[1].re + b[1].im), h * (b[1].im - b[1].re)};
  b[2] = cmul_mi(b[2]);
  b[3] = {h * (b[3].im - b[3].re), -h * (b[3].re + b[3].im)};
  dft4(a[0], a[1], a[2], a[3]);
  dft4(b[0], b[1], b[2], b[3]);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    v[2 * r] = a[r];
    v[2 * r + 1] = b[r];
  }
}

// One Stockham pass of radix R (8, 4 or 2) over the npg sequences of a
// group (sequence f at z + f*cp, complex units), stride ns = 8^.. so far:
// butterfly j reads s[j + m n/R] * w^(m k n/(R ns)) (k = j mod ns) and
// writes its DFT_R outputs to s[(j/ns) R ns + k + r ns].  NB bounds the
// butterflies per lane.
template <typename T, int R, int NB, int logn, int lns>
__device__ __forceinline__ void wave_pass(Cplx<T>* z, int cp, int npg, const Cplx<T>* __restrict__ tw) {
  using P = Pad<T>;
  constexpr int LR = R == 8 ? 3 : (R == 4 ? 2 : 1);
  const int lane = threadIdx.x & 63;
  constexpr int n = 1 << logn;
  constexpr int q = n >> LR;
  constexpr int ns = 1 << lns;
  const int nbf = q * npg;
  Cplx<T> v[NB][R];
#pragma unroll
  for (int it = 0; it < NB; ++it) {
    const int b = lane + it * 64;
    if (b < nbf) {
      const int f = b >> (logn - LR);
      const int j = b & (q - 1);
      const int k = j & (ns - 1);
      const int step = k << (logn - LR - lns);
      const Cplx<T>* s = z + f * cp;
      v[it][0] = s[P::cidx(j)];
#pragma unroll
      for (int m = 1; m < R; ++m) v[it][m] = cmul(s[P::cidx(j + m * q)], tw[m * step]);
    }
  }
  wave_sync();
#pragma unroll
  for (int it = 0; it < NB; ++it) {
    const int b = lane + it * 64;
    if (b < nbf) {
      if (R == 8) dft8(v[it]);
      if (R == 4) dft4(v[it][0], v[it][1], v[it][2], v[it][3]);
      if (R == 2) {
        const Cplx<T> t0 = v[it][0];
        v[it][0] = cadd(t0, v[it][1]);
        v[it][1] = csub(t0, v[it][1]);
      }
      const int f = b >> (logn - LR);
      const int j = b & (q - 1);
      const int k = j & (ns - 1);
      const int d0 = ((j >> lns) << (lns + LR)) + k;
      Cplx<T>* o = z + f * cp;
#pragma unroll
      for (int r = 0; r < R; ++r) o[P::cidx(d0 + r * ns)] = v[it][r];
    }
  }
  wave_sync();
}

// Stockham passes after the first: radix 8 while three or more factors of
// 2 are left, then one radix-4 or radix-2 pass (schedule fixed at compile
// time, so every index is a constant shift)
template <typename T, int E, int logn, int lns>
__device__ __forceinline__ void wave_passes(Cplx<T>* z, int cp, int npg, const Cplx<T>* __restrict__ tw) {
  if constexpr (lns + 3 <= logn) {
    wave_pass<T, 8, E / 8, logn, lns>(z, cp, npg, tw);
    wave_passes<T, E, logn, lns + 3>(z, cp, npg, tw);
  } else if constexpr (lns + 2 == logn) {
    wave_pass<T, 4, E / 4, logn, lns>(z, cp, npg, tw);
  } else if constexpr (lns + 1 == logn) {
    wave_pass<T, 2, E / 2, logn, lns>(z, cp, npg, tw);
  }
}

// Type-I sine transform of the npg row pairs of one group, by one wave.
// Pair f holds rows a (at g + f*ppitch) and b (at + rlen(n)), entry 0 = 0;
// on return entry p of each row holds S_p.  E = complex points per lane.
template <typename T, int E, int logn>
__device__ __forceinline__ void wave_dst(T* g, int npg, int ppitch, const Cplx<T>* __restrict__ tw,
                         const T* __restrict__ pre) {
  using P = Pad<T>;
  const int lane = threadIdx.x & 63;
  constexpr int n = 1 << logn;
  const int cp = ppitch / 2;
  Cplx<T>* z = reinterpret_cast<Cplx<T>*>(g);
  // A + first radix-8 pass: pre-twiddle straight into the butterfly inputs
  // (the first pass has no twiddles: k = 0)
  {
    constexpr int NB = E / 8;
    constexpr int q = n >> 3;
    const int nbf = q * npg;
    Cplx<T> v[NB][8];
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int b = lane + it * 64;
      if (b < nbf) {
        const int f = b >> (logn - 3);
        const int j = b & (q - 1);
        const T* ra = g + f * ppitch;
        const T* rb = ra + P::rlen(n);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int p = j + m * q;
          const T s = pre[p];
          const T a0 = ra[P::ridx(p)], b0 = rb[P::ridx(p)];
          const T a1 = p ? ra[P::ridx(n - p)] : T(0);
          const T b1 = p ? rb[P::ridx(n - p)] : T(0);
          v[it][m] = {s * (a0 + a1) + T(0.5) * (a0 - a1), s * (b0 + b1) + T(0.5) * (b0 - b1)};
        }
      }
    }
    wave_sync();
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int b = lane + it * 64;
      if (b < nbf) {
        dft8(v[it]);
        const int f = b >> (logn - 3);
        const int j = b & (q - 1);
        Cplx<T>* o = z + f * cp;
#pragma unroll
        for (int r = 0; r < 8; ++r) o[P::cidx(8 * j + r)] = v[it][r];
      }
    }
    wave_sync();
  }
  wave_passes<T, E, logn, 3>(z, cp, npg, tw);
  // C: unpack the two real spectra; even outputs directly, odd ones as the
  //    increments of the prefix sum
  {
    constexpr int NQ = E / 2;
    constexpr int h = n >> 1;
    const int nq = h * npg;
    T sa[NQ], ra_[NQ], sb[NQ], rb_[NQ];
#pragma unroll
    for (int it = 0; it < NQ; ++it) {
      const int e = lane + it * 64;
      if (e < nq) {
        const int f = e >> (logn - 1);
        const int q = e & (h - 1);
        const Cplx<T>* zz = z + f * cp;
        const Cplx<T> zq = zz[P::cidx(q)];
        const Cplx<T> zm = zz[P::cidx((n - q) & (n - 1))];
        sa[it] = q ? T(0.5) * (zm.im - zq.im) : T(0);
        sb[it] = q ? T(0.5) * (zq.re - zm.re) : T(0);
        ra_[it] = q ? T(0.5) * (zq.re + zm.re) : T(0.5) * zq.re;
        rb_[it] = q ? T(0.5) * (zq.im + zm.im) : T(0.5) * zq.im;
      }
    }
    wave_sync();
#pragma unroll
    for (int it = 0; it < NQ; ++it) {
      const int e = lane + it * 64;
      if (e < nq) {
        const int f = e >> (logn - 1);
        const int q = e & (h - 1);
        T* a = g + f * ppitch;
        T* b = a + P::rlen(n);
        a[P::ridx(2 * q)] = sa[it];
        a[P::ridx(2 * q + 1)] = ra_[it];
        b[P::ridx(2 * q)] = sb[it];
        b[P::ridx(2 * q + 1)] = rb_[it];
      }
    }
    wave_sync();
  }
  // D: odd outputs = inclusive prefix sums of the odd entries, per row.
  //    The 2*npg rows of the group hold n/2 odd entries each; a lane takes
  //    c = E/... consecutive entries of one row, the lanes of a row scan
  //    their chunk totals with shuffles.
  {
    constexpr int h = n >> 1;
    const int total = 2 * npg * h;              // odd entries in the group
    const int c = total >= 64 ? total / 64 : 1; // entries per lane
    const int active = total / c;
    const int tpr = h / c;                      // lanes per row (power of 2, <= 64)
    T loc[E];
    T run = T(0);
    int row = 0, q0 = 0;
    if (lane < active) {
      row = (lane * c) / h;
      q0 = (lane * c) % h;
      T* r = g + (row >> 1) * ppitch + (row & 1) * P::rlen(n);
#pragma unroll
      for (int t = 0; t < E; ++t) {
        if (t < c) {
          run += r[P::ridx(2 * (q0 + t) + 1)];
          loc[t] = run;
        }
      }
    }
    T incl = run;
    for (int off = 1; off < tpr; off <<= 1) {
      const T o = __shfl_up(incl, off, 64);
      if ((lane & (tpr - 1)) >= off) incl += o;
    }
    const T excl = incl - run;
    wave_sync();
    if (lane < active) {
      T* r = g + (row >> 1) * ppitch + (row & 1) * P::rlen(n);
#pragma unroll
      for (int t = 0; t < E; ++t)
        if (t < c) r[P::ridx(2 * (q0 + t) + 1)] = loc[t] + excl;
    }
    wave_sync();
  }
}

// Type-I sine transform of nrow rows (nrow even) of length n = 2^logn held
// in LDS; pair f = rows (2f, 2f+1) occupies buf[f*ppitch .. f*ppitch + 2n)
// (row 2f first).  Entry 0 of every input row must be 0; on output entry p
// holds S_p (entry 0 = 0).  Groups of max(1, 512/n) pairs are handed to the
// workgroup's waves in turn; ends with a workgroup barrier.
template <typename T, int LOGN>
__device__ __forceinline__ void block_dst(T* buf, int logn, int nrow, int ppitch,
                                          const Cplx<T>* __restrict__ tw,
                                          const T* __restrict__ pre) {
  constexpr int n = 1 << LOGN;
  constexpr int per = n >= 512 ? 1 : 512 / n;
  constexpr int E = n <= 512 ? 8 : n / 64;
  (void)logn;
  const int npair = nrow >> 1;
  const int ngroup = (npair + per - 1) / per;
  const int wave = threadIdx.x >> 6;
  const int nwave = blockDim.x >> 6;
  for (int gi = wave; gi < ngroup; gi += nwave) {
    const int npg = min(per, npair - gi * per);
    wave_dst<T, E, LOGN>(buf + static_cast<size_t>(gi) * per * ppitch, npg, ppitch, tw, pre);
  }
  __syncthreads();
}

// Runs f(std::integral_constant<int, log2 n>) for the transform length n
// (a power of two in [16, 2048]); every kernel is instantiated per length.
template <typename F>
void with_logn(int n, F&& f) {
  switch (n) {
    case 16: f(std::integral_constant<int, 4>{}); break;
    case 32: f(std::integral_constant<int, 5>{}); break;
    case 64: f(std::integral_constant<int, 6>{}); break;
    case 128: f(std::integral_constant<int, 7>{}); break;
    case 256: f(std::integral_constant<int, 8>{}); break;
    case 512: f(std::integral_constant<int, 9>{}); break;
    case 1024: f(std::integral_constant<int, 10>{}); break;
    case 2048: f(std::integral_constant<int, 11>{}); break;
    default: throw std::invalid_argument("transform length must be a power of two in [16, 2048]");
  }
}

template <typename T>
__host__ __device__ inline size_t table_bytes(int n) {
  return static_cast<size_t>(n) * (sizeof(Cplx<T>) + sizeof(T));
}

// Busy waves per workgroup of a transform pass: each wave transforms a group
// of max(1, 512/n) row pairs.  The QSP_ROW_WAVES / QSP_COL_WAVES environment
// variables (1, 2 or 4) override the defaults for tuning.
inline int pass_waves(const char* env, int dflt) {
  if (const char* e = std::getenv(env)) {
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4) return v;
  }
  return dflt;
}

template <typename T>
inline size_t pass_lds(int rows, int n) {
  return static_cast<size_t>(rows / 2) * Pad<T>::pitch(n) * sizeof(T) + table_bytes<T>(n) +
         static_cast<size_t>(n) * sizeof(double);
}

// columns per column-pass workgroup (even, at most nx, within 80 KiB of LDS).
// One busy wave (one column pair) per workgroup up to 512 rows (FP32) or
// 256 rows (FP64); beyond, two, whose four-column strips halve the strided
// row segments each workgroup reads (measured from HIP graphs: 8 % off a
// 1024^2 time step in FP32, 2 % off the 512^2 box in FP64).
template <typename T>
inline int col_strip(int nx, int ny, int nfield) {
  (void)nfield;
  const int per = ny >= 512 ? 1 : 512 / ny;
  const int waves = ny >= (sizeof(T) == 8 ? 512 : 1024) ? 2 : 1;
  int w = 2 * per * pass_waves("QSP_COL_WAVES", waves);
  if (const char* e = std::getenv("QSP_COL_W")) {   // tuning override
    const int v = std::atoi(e);
    if (v >= 2 && (v & (v - 1)) == 0) w = v;
  }
  if (w > nx) w = nx;
  while (w > 2 && pass_lds<T>(w, ny) > 81920) w >>= 1;   // two workgroups per CU
  return w;
}

// Copies an axis' twiddle and pre-twiddle tables into LDS right after the
// workgroup's data region, so the FFT stages never wait on global memory.
template <typename T>
__device__ inline void stage_tables(const AxisTables<T>& t, int n, unsigned char* base,
                                    const Cplx<T>*& tw, const T*& pre) {
  Cplx<T>* stw = reinterpret_cast<Cplx<T>*>(base);
  T* spre = reinterpret_cast<T*>(base + n * sizeof(Cplx<T>));
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    stw[i] = t.tw[i];
    spre[i] = t.pre[i];
  }
  tw = stw;
  pre = spre;
}

// clears the planes of z, workgroup `bid` of `nblk` taking every nblk-th
// block of kBlock elements
__device__ inline void zero_job(const ZeroJob& z, size_t bid, size_t nblk) {
  if (z.count == 0) return;
  const size_t stride = nblk * blockDim.x;
  const size_t start = bid * blockDim.x + threadIdx.x;
  for (int c = 0; c < z.count; ++c)
    for (size_t i = start; i < z.n; i += stride) z.p[c][i] = 0.0;
}

template <typename T>
__device__ inline void guess_job(const GuessJob<T>& q, size_t n) {
  if (!q.ctr) return;
  const size_t stride = static_cast<size_t>(gridDim.x) * gridDim.y * blockDim.x;
  const size_t bid = static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x;
  if (bid == 0 && threadIdx.x == 0) {
    q.ctr->pc_done = 0u;
    q.ctr->pc_iters = 0u;
    q.ctr->pc_resid = 0.0;
  }
  for (size_t i = bid * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T vx = T(2) * q.bx1[i] - q.bx2[i];
    const T vy = T(2) * q.by1[i] - q.by2[i];
    q.bx[i] = vx;
    q.by[i] = vy;
    if (q.tape_bx) {
      q.tape_bx[i] = vx;
      q.tape_by[i] = vy;
    }
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Neighbouring column strips share cache lines, so strip s is given to
// the workgroup that lands on XCD (s / per) - keeping each XCD on one
// contiguous range of strips.
__device__ inline int xcd_strip(int b, int nstrip) {
  if (nstrip < 8 || (nstrip & 7)) return b;
  const int per = nstrip >> 3;
  return (b & 7) * per + (b >> 3);
}

// Workgroups per CU the transform kernels are compiled for: four (<= 128
// VGPRs) while a lane holds at most 8 FP32 complex points, fewer for the
// long FP64 transforms whose register arrays would otherwise spill.
constexpr int dst_blocks_per_cu(int logn, int tsize) {
  const int u = (logn <= 9 ? 8 : (1 << logn) / 64) * tsize / 4;
  return u <= 8 ? 4 : (u <= 16 ? 2 : 1);
}

// Calls f(e) for the workgroup's elements e = threadIdx.x + it*kBlock,
// e < total.  The whole multiples of kBlock run as unrolled straight-line
// chunks of up to 8, so with a branch-free f the global loads of a chunk are
// in flight together instead of one load latency per element.
template <int CH, typename F>
__device__ __forceinline__ void elem_chunk(int& it, F& f) {
#pragma unroll
  for (int u = 0; u < CH; ++u) f(static_cast<int>(threadIdx.x) + (it + u) * kBlock);
  it += CH;
}

template <typename F>
__device__ __forceinline__ void for_elems(int total, F&& f) {
  const int nit = total / kBlock;   // uniform across the workgroup
  int it = 0;
  while (it + 8 <= nit) elem_chunk<8>(it, f);
  if (nit & 4) elem_chunk<4>(it, f);
  if (nit & 2) elem_chunk<2>(it, f);
  if (nit & 1) elem_chunk<1>(it, f);
  for (int e = nit * kBlock + static_cast<int>(threadIdx.x); e < total; e += kBlock) f(e);
}



// Source assembly (FP64) + forward DST along x of row block bxi of field
// fld (0 Bx, 1 By) of the Bx/By predictor-corrector.
template <typename T, int LOGN>
__device__ __forceinline__ void src_bxby_block(const Geom& g, const SrcBxBy<T>& a,
                                               const AxisTables<T>& tx, int bxi, int fld,
                                               unsigned char* smem_raw) {
  __syncthreads();   // the workgroup's previous use of LDS is complete
  T* buf = reinterpret_cast<T*>(smem_raw);
  const int n = g.nx;
  const int R = g.rr;
  const int ppitch = Pad<T>::pitch(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables(tx, n, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int j0 = bxi * R;
  const double ihx = 0.5 / g.hx, ihy = 0.5 / g.hy;
  const double idz = 0.5 / a.dzeta;
  const int lx = g.lx;
  const double amp = a.beam_amp;
  for_elems(R * n, [&](int e) {
    const int r = e >> lx, i = e & (n - 1);
    const int j = j0 + r;
    const int o = j * n + i;
    double s;
    if (fld == 0) {
      // -d_y Jz + (Jy_{k-1} - Jy_{k+1}) / (2 dzeta) - shift * Bx_old
      const int js = j > 0 ? j - 1 : 0;
      const double zs = a.jz[js * n + i], zn = a.jz[(j + 1 < g.ny ? j + 1 : j) * n + i];
      const double yp = a.jy_prev[o], yt = a.jy_next[o];
      const double bo = static_cast<double>(a.bx[o]);
      const double gx = a.bgx[i], gs = a.bgy[js], gn = a.bgy[j + 1];
      const double jz_s = zs - amp * gx * gs;
      const double jz_n = j + 1 < g.ny ? zn - amp * gx * gn : 0.0;
      s = -(jz_n - jz_s) * ihy + (yp - yt) * idz - a.shift * bo;
    } else {
      // d_x Jz - (Jx_{k-1} - Jx_{k+1}) / (2 dzeta) - shift * By_old
      const int iw = i > 0 ? i - 1 : 0;
      const double zw = a.jz[j * n + iw], ze = a.jz[j * n + (i + 1 < n ? i + 1 : i)];
      const double xp = a.jx_prev[o], xt = a.jx_next[o];
      const double bo = static_cast<double>(a.by[o]);
      const double gy = a.bgy[j], gw = a.bgx[iw], ge = a.bgx[i + 1];
      const double jz_w = zw - amp * gw * gy;
      const double jz_e = i + 1 < n ? ze - amp * ge * gy : 0.0;
      s = (jz_e - jz_w) * ihx - (xp - xt) * idz - a.shift * bo;
    }
    buf[Pad<T>::rpos(n, ppitch, r, i)] = static_cast<T>((i > 0 && j > 0) ? s : 0.0);
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  T* out = a.out + static_cast<size_t>(fld) * g.nx * g.ny;
  for_elems(R * n, [&](int e) {
    const int r = e >> lx, i = e & (n - 1);
    out[(j0 + r) * n + i] = buf[Pad<T>::rpos(n, ppitch, r, i)];
  });
}

// DST along y, eigenvalue division, inverse DST along y (and -d_y for
// field 0 when requested) of column strip `strip` of field fld.
template <typename T, int LOGN>
__device__ __forceinline__ void col_block(const Geom& g, const ColArgs<T>& a,
                                          const AxisTables<T>& ty, const double* __restrict__ lamx,
                                          int strip, int fld, unsigned char* smem_raw) {
  __syncthreads();   // the workgroup's previous use of LDS is complete
  T* buf = reinterpret_cast<T*>(smem_raw);
  const int ny = g.ny, nx = g.nx;
  const int W = a.w;
  const int ppitch = Pad<T>::pitch(ny);
  const int p0 = strip * W;
  unsigned char* tbase = smem_raw + static_cast<size_t>(W / 2) * ppitch * sizeof(T);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables(ty, ny, tbase, tw, pre);
  double* slam = reinterpret_cast<double*>(tbase + table_bytes<T>(ny));
  for (int i = threadIdx.x; i < ny; i += blockDim.x) slam[i] = ty.lam[i];
  const size_t plane = static_cast<size_t>(nx) * ny;
  const T* in = a.in + fld * plane;
  const int lw = 31 - __clz(W), ly = g.ly;
  for_elems(W * ny, [&](int e) {
    const int c = e & (W - 1), j = e >> lw;
    buf[Pad<T>::rpos(ny, ppitch, c, j)] = in[j * nx + p0 + c];
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.ly, W, ppitch, tw, pre);
  const double shift = a.shift[fld];
  const double norm = 4.0 / (static_cast<double>(nx) * ny);
  for_elems(W * ny, [&](int e) {
    const int c = e >> ly, q = e & (ny - 1);
    const int p = p0 + c;
    T* r = buf + Pad<T>::rpos(ny, ppitch, c, 0);
    const double den = lamx[p] + slam[q] - shift;
    const int iq = Pad<T>::ridx(q);
    const double v = static_cast<double>(r[iq]) * norm / den;
    r[iq] = (p > 0 && q > 0) ? static_cast<T>(v) : T(0);
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.ly, W, ppitch, tw, pre);
  T* out = a.out + fld * plane;
  T* out_dy = (fld == 0) ? a.out_dy : nullptr;
  const T mihy = static_cast<T>(-0.5 / g.hy);
  for_elems(W * ny, [&](int e) {
    const int c = e & (W - 1), j = e >> lw;
    const T* r = buf + Pad<T>::rpos(ny, ppitch, c, 0);
    out[j * nx + p0 + c] = r[Pad<T>::ridx(j)];
    if (out_dy) {
      const T up = r[Pad<T>::ridx(j + 1 < ny ? j + 1 : j)], dn = r[Pad<T>::ridx(j > 0 ? j - 1 : 0)];
      const T d = mihy * ((j + 1 < ny ? up : T(0)) - dn);
      out_dy[j * nx + p0 + c] = j > 0 ? d : T(0);
    }
  });
}

// Predictor-corrector epilogue: B_new from the inverse transform, FP64 sums
// of |B_new - B_old|^2 and |B_new|^2, B_old overwritten by B_new in place.
// Each workgroup leaves its two sums in a.partial; the next trial push (or
// the real push after the last iteration) forms the relative change and
// decides convergence.
template <typename T, int LOGN>
__device__ __forceinline__ void row_inv_pc_block(const Geom& g, const PCArgs<T>& a,
                                                 const AxisTables<T>& tx, int bxi, int fld,
                                                 unsigned char* smem_raw) {
  __syncthreads();   // the workgroup's previous use of LDS is complete
  T* buf = reinterpret_cast<T*>(smem_raw);
  const int n = g.nx;
  const int R = g.rr;
  const int ppitch = Pad<T>::pitch(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables(tx, n, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int j0 = bxi * R;
  const T* in = a.in + static_cast<size_t>(fld) * g.nx * g.ny;
  const int lx = g.lx;
  for_elems(R * n, [&](int e) {
    const int r = e >> lx, i = e & (n - 1);
    buf[Pad<T>::rpos(n, ppitch, r, i)] = in[(j0 + r) * n + i];
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  T* b = fld == 0 ? a.bx : a.by;
  T* tp = fld == 0 ? a.tape_bx : a.tape_by;
  double dsum = 0.0, nsum = 0.0;
  for_elems(R * n, [&](int e) {
    const int r = e >> lx, i = e & (n - 1);
    const int j = j0 + r;
    const T v = buf[Pad<T>::rpos(n, ppitch, r, i)];
    const T u = j > 0 ? v : T(0);
    const double old = static_cast<double>(b[j * n + i]);
    const double d = static_cast<double>(u) - old;
    dsum += d * d;
    nsum += static_cast<double>(u) * static_cast<double>(u);
    b[j * n + i] = u;
    if (tp) tp[j * n + i] = u;
  });
  double v[2] = {dsum, nsum};
  partials::store<2>(v, a.partial, fld * (g.ny / R) + bxi);
}

}  // namespace dst_detail

// rows per row-pass workgroup (even, at most ny, within 144 KiB of LDS).
// Up to 512 columns one busy wave per workgroup (more, smaller workgroups
// fill the chip; measured best from HIP graphs at 64^2 and 512^2), above
// two in FP32 and four in FP64 (measured at 1024^2).
template <typename T>
int row_rows(int nx, int ny) {
  const int per = nx >= 512 ? 1 : 512 / nx;
  const int waves = nx <= 512 ? 1 : (sizeof(T) == 8 ? 4 : 2);
  int r = 2 * per * dst_detail::pass_waves("QSP_ROW_WAVES", waves);
  if (r > ny) r = ny;
  while (r > 2 && dst_detail::pass_lds<T>(r, nx) > 147456) r >>= 1;
  return r;
}

}  // namespace qsp
