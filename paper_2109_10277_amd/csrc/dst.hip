// Batched 2D Dirichlet Poisson / Helmholtz solves with type-I sine transforms
// (fast Poisson solver of HiPACE++, arXiv:2109.10277 Sec. III.B), written for
// gfx950: every 1D transform runs inside LDS, two real rows packed into one
// complex FFT (Stockham radix-4/2), with a pre-twiddle that reduces the
// DST-I of length n-1 to a complex FFT of length n per row pair.
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
#include <cstdlib>
#include <stdexcept>

#include "common.hpp"
#include "kernels.hpp"

namespace qsp {

namespace {

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

// In-place Stockham FFT (forward, e^{-2 pi i jk/n}) of `nfft` sequences of
// length n = 2^logn; sequence f starts at buf + f*pitch (complex units).
// tw[m] = e^{-2 pi i m / n}.  MAXB bounds the radix-4 butterflies per thread.
template <typename T, int MAXB>
__device__ void block_fft(Cplx<T>* buf, int logn, int nfft, int pitch,
                          const Cplx<T>* __restrict__ tw) {
  using P = Pad<T>;
  const int n = 1 << logn;
  const int tid = threadIdx.x;
  int ns = 1;
  int lns = 0;
  while (lns + 2 <= logn) {
    const int q = n >> 2;             // butterflies per sequence
    const int nbf = q * nfft;
    Cplx<T> v[MAXB][4];
#pragma unroll
    for (int it = 0; it < MAXB; ++it) {
      const int b = tid + it * kBlock;
      if (b < nbf) {
        const int f = b >> (logn - 2);
        const int j = b & (q - 1);
        const int k = j & (ns - 1);
        Cplx<T>* s = buf + f * pitch;
        const int step = k << (logn - 2 - lns);   // k * n / (4 ns)
        v[it][0] = s[P::cidx(j)];
        v[it][1] = cmul(s[P::cidx(j + q)], tw[step]);
        v[it][2] = cmul(s[P::cidx(j + 2 * q)], tw[2 * step]);
        v[it][3] = cmul(s[P::cidx(j + 3 * q)], tw[3 * step]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXB; ++it) {
      const int b = tid + it * kBlock;
      if (b < nbf) {
        const Cplx<T> a0 = v[it][0], a1 = v[it][1], a2 = v[it][2], a3 = v[it][3];
        const Cplx<T> s02 = {a0.re + a2.re, a0.im + a2.im};
        const Cplx<T> d02 = {a0.re - a2.re, a0.im - a2.im};
        const Cplx<T> s13 = {a1.re + a3.re, a1.im + a3.im};
        const Cplx<T> d13 = {a1.re - a3.re, a1.im - a3.im};
        const int f = b >> (logn - 2);
        const int j = b & (q - 1);
        const int d0 = ((j >> lns) << (lns + 2)) + (j & (ns - 1));
        Cplx<T>* o = buf + f * pitch;
        o[P::cidx(d0)] = {s02.re + s13.re, s02.im + s13.im};
        o[P::cidx(d0 + ns)] = {d02.re + d13.im, d02.im - d13.re};       // a0 - i a1 - a2 + i a3
        o[P::cidx(d0 + 2 * ns)] = {s02.re - s13.re, s02.im - s13.im};
        o[P::cidx(d0 + 3 * ns)] = {d02.re - d13.im, d02.im + d13.re};   // a0 + i a1 - a2 - i a3
      }
    }
    __syncthreads();
    ns <<= 2;
    lns += 2;
  }
  if (lns < logn) {  // one radix-2 stage (ns = n/2)
    const int h = n >> 1;
    const int nbf = h * nfft;
    Cplx<T> v[2 * MAXB][2];
#pragma unroll
    for (int it = 0; it < 2 * MAXB; ++it) {
      const int b = tid + it * kBlock;
      if (b < nbf) {
        const int f = b >> (logn - 1);
        const int j = b & (h - 1);
        Cplx<T>* s = buf + f * pitch;
        v[it][0] = s[P::cidx(j)];
        v[it][1] = cmul(s[P::cidx(j + h)], tw[j]);    // k = j, step n/(2 ns) = 1
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 2 * MAXB; ++it) {
      const int b = tid + it * kBlock;
      if (b < nbf) {
        const int f = b >> (logn - 1);
        const int j = b & (h - 1);
        Cplx<T>* o = buf + f * pitch;
        o[P::cidx(j)] = {v[it][0].re + v[it][1].re, v[it][0].im + v[it][1].im};
        o[P::cidx(j + h)] = {v[it][0].re - v[it][1].re, v[it][0].im - v[it][1].im};
      }
    }
    __syncthreads();
  }
}

// Inclusive prefix sum over the odd entries (1, 3, ..., n-1) of each of the
// nrow rows (row r at buf + (r/2)*ppitch + (r&1)*n, real units).
template <typename T, int MAXC>
__device__ void block_odd_scan(T* buf, int logn, int nrow, int ppitch, T* wsum) {
  using P = Pad<T>;
  const int n = 1 << logn;
  const int half = n >> 1;
  const int total = nrow * half;
  const int tid = threadIdx.x;
  // chunk of c consecutive odd entries of one row per thread
  const int c = total >= kBlock ? total / kBlock : 1;
  const int active = total / c;                // threads holding a chunk
  const int tpr = half / c;                    // threads per row (power of 2)
  T loc[MAXC];
  T run = 0;
  int row = 0, q0 = 0;
  if (tid < active) {
    row = (tid * c) / half;
    q0 = (tid * c) % half;
    T* r = buf + (row >> 1) * ppitch + (row & 1) * P::rlen(n);
#pragma unroll
    for (int t = 0; t < MAXC; ++t) {
      if (t < c) {
        run += r[P::ridx(2 * (q0 + t) + 1)];
        loc[t] = run;
      }
    }
  }
  // inclusive scan of the chunk totals across the threads of each row
  const int lane = tid & 63;
  const int width = tpr < 64 ? tpr : 64;
  T incl = run;
  for (int off = 1; off < width; off <<= 1) {
    const T o = __shfl_up(incl, off, 64);
    if ((lane & (width - 1)) >= off) incl += o;
  }
  if (tpr > 64) {
    const int wave = tid >> 6;
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    const int first = (wave / (tpr >> 6)) * (tpr >> 6);
    T add = 0;
    for (int w = first; w < wave; ++w) add += wsum[w];
    incl += add;
  }
  const T excl = incl - run;
  __syncthreads();   // every thread has read its inputs
  if (tid < active) {
    T* r = buf + (row >> 1) * ppitch + (row & 1) * P::rlen(n);
#pragma unroll
    for (int t = 0; t < MAXC; ++t)
      if (t < c) r[P::ridx(2 * (q0 + t) + 1)] = loc[t] + excl;
  }
  __syncthreads();
}

// Type-I sine transform of nrow rows (nrow even) of length n = 2^logn held
// in LDS; pair f = rows (2f, 2f+1) occupies buf[f*ppitch .. f*ppitch + 2n)
// (row 2f first).  Entry 0 of every input row must be 0; on output entry p
// holds S_p (entry 0 = 0).  MAXC bounds the complex elements per thread.
template <typename T, int MAXC>
__device__ void block_dst(T* buf, int logn, int nrow, int ppitch,
                          const Cplx<T>* __restrict__ tw, const T* __restrict__ pre,
                          T* wsum) {
  using P = Pad<T>;
  const int n = 1 << logn;
  const int tid = threadIdx.x;
  const int npair = nrow >> 1;
  const int ncplx = npair * n;
  // A: pre-twiddle into packed complex rows
  {
    T ya[MAXC], yb[MAXC];
#pragma unroll
    for (int it = 0; it < MAXC; ++it) {
      const int e = tid + it * kBlock;
      if (e < ncplx) {
        const int f = e >> logn;
        const int j = e & (n - 1);
        const T* ra = buf + f * ppitch;
        const T* rb = ra + P::rlen(n);
        const T s = pre[j];
        const T a0 = ra[P::ridx(j)], b0 = rb[P::ridx(j)];
        const T a1 = j ? ra[P::ridx(n - j)] : T(0);
        const T b1 = j ? rb[P::ridx(n - j)] : T(0);
        ya[it] = s * (a0 + a1) + T(0.5) * (a0 - a1);
        yb[it] = s * (b0 + b1) + T(0.5) * (b0 - b1);
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXC; ++it) {
      const int e = tid + it * kBlock;
      if (e < ncplx) {
        const int f = e >> logn;
        const int j = e & (n - 1);
        Cplx<T>* z = reinterpret_cast<Cplx<T>*>(buf + f * ppitch);
        z[P::cidx(j)] = {ya[it], yb[it]};
      }
    }
    __syncthreads();
  }
  // B: complex FFTs of the packed pairs
  block_fft<T, (MAXC + 3) / 4>(reinterpret_cast<Cplx<T>*>(buf), logn, npair,
                               ppitch / 2, tw);
  // C: unpack the two real spectra; even outputs directly, odd ones as the
  //    increments of the prefix sum
  {
    constexpr int MQ = (MAXC + 1) / 2;
    T sa[MQ], ra[MQ], sb[MQ], rb[MQ];
    const int nq = npair * (n >> 1);
#pragma unroll
    for (int it = 0; it < MQ; ++it) {
      const int e = tid + it * kBlock;
      if (e < nq) {
        const int f = e >> (logn - 1);
        const int q = e & ((n >> 1) - 1);
        const Cplx<T>* z = reinterpret_cast<const Cplx<T>*>(buf + f * ppitch);
        const Cplx<T> zq = z[P::cidx(q)];
        const Cplx<T> zm = z[P::cidx((n - q) & (n - 1))];
        sa[it] = q ? T(0.5) * (zm.im - zq.im) : T(0);
        sb[it] = q ? T(0.5) * (zq.re - zm.re) : T(0);
        ra[it] = q ? T(0.5) * (zq.re + zm.re) : T(0.5) * zq.re;
        rb[it] = q ? T(0.5) * (zq.im + zm.im) : T(0.5) * zq.im;
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MQ; ++it) {
      const int e = tid + it * kBlock;
      if (e < nq) {
        const int f = e >> (logn - 1);
        const int q = e & ((n >> 1) - 1);
        T* a = buf + f * ppitch;
        T* b = a + P::rlen(n);
        a[P::ridx(2 * q)] = sa[it];
        a[P::ridx(2 * q + 1)] = ra[it];
        b[P::ridx(2 * q)] = sb[it];
        b[P::ridx(2 * q + 1)] = rb[it];
      }
    }
    __syncthreads();
  }
  // D: odd outputs
  block_odd_scan<T, MAXC>(buf, logn, nrow, ppitch, wsum);
}

// rows per row-pass workgroup: 2048 elements (at least two rows), at most ny
__host__ __device__ inline int row_block_rows(int nx, int ny) {
  const int r = nx >= 1024 ? 2 : 2048 / nx;
  return r < ny ? r : ny;
}

// columns per column-pass workgroup: at most a 32 KiB LDS strip and at most
// 16 columns, and narrow enough that the pass has >= 512 workgroups
template <typename T>
inline int col_strip(int nx, int ny, int nfield) {
  const int lim = 32768 / static_cast<int>(sizeof(T));
  int w = 16;
  while (w > 2 && (w * ny > lim || (nx / w) * nfield < 512)) w >>= 1;
  if (const char* e = std::getenv("QSP_COL_W")) {   // tuning override
    const int v = std::atoi(e);
    if (v >= 2 && v <= 16 && (v & (v - 1)) == 0 && v * ny <= lim) w = v;
  }
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

template <typename T>
__host__ __device__ inline size_t table_bytes(int n) {
  return static_cast<size_t>(n) * (sizeof(Cplx<T>) + sizeof(T));
}

__device__ inline void zero_job(const ZeroJob& z) {
  if (z.count == 0) return;
  const size_t stride = static_cast<size_t>(gridDim.x) * gridDim.y * blockDim.x;
  const size_t start = (static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x) * blockDim.x +
                       threadIdx.x;
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

constexpr int kRowMaxC = 8;    // n <= 2048: 2 rows x 2048 / 512 complex per thread
constexpr int kColMaxC = 16;
constexpr int kRowMaxE = 16;   // row-pass elements per thread (2 rows of 2048)
constexpr int kColMaxE = 32;   // column-pass elements per thread (32 KiB strip)

}  // namespace

// ---------------------------------------------------------------------------
// P1: sources + forward DST along x
// ---------------------------------------------------------------------------

// field ids of the psi / Ez / Bz batch
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_src_fwd_pez(Geom g, SrcPEZ<T> a, AxisTables<T> tx) {
  extern __shared__ unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  __shared__ T wsum[4];
  const int n = g.nx;
  const int R = row_block_rows(n, g.ny);
  const int ppitch = Pad<T>::pitch(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables(tx, n, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int j0 = blockIdx.x * R;
  const int fld = blockIdx.y;   // 0 psi, 1 Ez, 2 Bz
  const double ihx = 0.5 / g.hx, ihy = 0.5 / g.hy;
#pragma unroll
  for (int it = 0; it < kRowMaxE; ++it) {
    const int e = threadIdx.x + it * kBlock;
    if (e >= R * n) break;
    const int r = e / n, i = e % n;
    const int j = j0 + r;
    double s = 0.0;
    if (i > 0 && j > 0) {
      const int o = j * n + i;
      if (fld == 0) {
        s = -(a.rho_mjz[o] + a.n0);
      } else {
        const double jx_e = i + 1 < n ? a.jx[o + 1] : 0.0, jx_w = a.jx[o - 1];
        const double jy_e = i + 1 < n ? a.jy[o + 1] : 0.0, jy_w = a.jy[o - 1];
        const double jx_n = j + 1 < g.ny ? a.jx[o + n] : 0.0, jx_s = a.jx[o - n];
        const double jy_n = j + 1 < g.ny ? a.jy[o + n] : 0.0, jy_s = a.jy[o - n];
        if (fld == 1)
          s = (jx_e - jx_w) * ihx + (jy_n - jy_s) * ihy;
        else
          s = (jx_n - jx_s) * ihy - (jy_e - jy_w) * ihx;
      }
    }
    buf[Pad<T>::rpos(n, ppitch, r, i)] = static_cast<T>(s);
  }
  __syncthreads();
  block_dst<T, kRowMaxC>(buf, g.lx, R, ppitch, tw, pre, wsum);
  T* out = a.out + static_cast<size_t>(fld) * g.nx * g.ny;
#pragma unroll
  for (int it = 0; it < kRowMaxE; ++it) {
    const int e = threadIdx.x + it * kBlock;
    if (e >= R * n) break;
    const int r = e / n, i = e % n;
    out[(j0 + r) * n + i] = buf[Pad<T>::rpos(n, ppitch, r, i)];
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_src_fwd_bxby(Geom g, SrcBxBy<T> a, AxisTables<T> tx, const DevCounters* ctr) {
  if (ctr->pc_done) return;
  extern __shared__ unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  __shared__ T wsum[4];
  const int n = g.nx;
  const int R = row_block_rows(n, g.ny);
  const int ppitch = Pad<T>::pitch(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables(tx, n, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int j0 = blockIdx.x * R;
  const int fld = blockIdx.y;   // 0 Bx, 1 By
  const double ihx = 0.5 / g.hx, ihy = 0.5 / g.hy;
  const double idz = 0.5 / a.dzeta;
#pragma unroll
  for (int it = 0; it < kRowMaxE; ++it) {
    const int e = threadIdx.x + it * kBlock;
    if (e >= R * n) break;
    const int r = e / n, i = e % n;
    const int j = j0 + r;
    double s = 0.0;
    if (i > 0 && j > 0) {
      const int o = j * n + i;
      if (fld == 0) {
        // -d_y Jz + (Jy_{k-1} - Jy_{k+1}) / (2 dzeta) - shift * Bx_old
        double jz_n = 0.0, jz_s = a.jz[o - n];
        if (j + 1 < g.ny) jz_n = a.jz[o + n];
        if (a.beam_amp != 0.0) {
          jz_s -= a.beam_amp * a.bgx[i] * a.bgy[j - 1];
          if (j + 1 < g.ny) jz_n -= a.beam_amp * a.bgx[i] * a.bgy[j + 1];
        }
        s = -(jz_n - jz_s) * ihy + (a.jy_prev[o] - a.jy_next[o]) * idz -
            a.shift * static_cast<double>(a.bx[o]);
      } else {
        double jz_e = 0.0, jz_w = a.jz[o - 1];
        if (i + 1 < n) jz_e = a.jz[o + 1];
        if (a.beam_amp != 0.0) {
          jz_w -= a.beam_amp * a.bgx[i - 1] * a.bgy[j];
          if (i + 1 < n) jz_e -= a.beam_amp * a.bgx[i + 1] * a.bgy[j];
        }
        s = (jz_e - jz_w) * ihx - (a.jx_prev[o] - a.jx_next[o]) * idz -
            a.shift * static_cast<double>(a.by[o]);
      }
    }
    buf[Pad<T>::rpos(n, ppitch, r, i)] = static_cast<T>(s);
  }
  __syncthreads();
  block_dst<T, kRowMaxC>(buf, g.lx, R, ppitch, tw, pre, wsum);
  T* out = a.out + static_cast<size_t>(fld) * g.nx * g.ny;
#pragma unroll
  for (int it = 0; it < kRowMaxE; ++it) {
    const int e = threadIdx.x + it * kBlock;
    if (e >= R * n) break;
    const int r = e / n, i = e % n;
    out[(j0 + r) * n + i] = buf[Pad<T>::rpos(n, ppitch, r, i)];
  }
}

// ---------------------------------------------------------------------------
// P2: column strip solve
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_col_solve(Geom g, ColArgs<T> a, AxisTables<T> ty, const double* __restrict__ lamx,
            const DevCounters* ctr) {
  if (a.honor_done && ctr->pc_done) return;
  zero_job(a.zero);
  extern __shared__ unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  __shared__ T wsum[4];
  const int ny = g.ny, nx = g.nx;
  const int W = a.w;
  const int ppitch = Pad<T>::pitch(ny);
  const int p0 = xcd_strip(blockIdx.x, gridDim.x) * W;
  unsigned char* tbase = smem_raw + static_cast<size_t>(W / 2) * ppitch * sizeof(T);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables(ty, ny, tbase, tw, pre);
  double* slam = reinterpret_cast<double*>(tbase + table_bytes<T>(ny));
  for (int i = threadIdx.x; i < ny; i += blockDim.x) slam[i] = ty.lam[i];
  const int fld = blockIdx.y;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const T* in = a.in + fld * plane;
#pragma unroll
  for (int it = 0; it < kColMaxE; ++it) {
    const int e = threadIdx.x + it * kBlock;
    if (e >= W * ny) break;
    const int c = e % W, j = e / W;
    buf[Pad<T>::rpos(ny, ppitch, c, j)] = in[j * nx + p0 + c];
  }
  __syncthreads();
  block_dst<T, kColMaxC>(buf, g.ly, W, ppitch, tw, pre, wsum);
  const double shift = a.shift[fld];
  const double norm = 4.0 / (static_cast<double>(nx) * ny);
#pragma unroll
  for (int it = 0; it < kColMaxE; ++it) {
    const int e = threadIdx.x + it * kBlock;
    if (e >= W * ny) break;
    const int c = e / ny, q = e % ny;
    const int p = p0 + c;
    T* r = buf + Pad<T>::rpos(ny, ppitch, c, 0);
    const double den = lamx[p] + slam[q] - shift;
    const int iq = Pad<T>::ridx(q);
    r[iq] = (p > 0 && q > 0) ? static_cast<T>(static_cast<double>(r[iq]) * norm / den) : T(0);
  }
  __syncthreads();
  block_dst<T, kColMaxC>(buf, g.ly, W, ppitch, tw, pre, wsum);
  T* out = a.out + fld * plane;
  const bool dy = (fld == 0) && a.out_dy != nullptr;
  const T mihy = static_cast<T>(-0.5 / g.hy);
#pragma unroll
  for (int it = 0; it < kColMaxE; ++it) {
    const int e = threadIdx.x + it * kBlock;
    if (e >= W * ny) break;
    const int c = e % W, j = e / W;
    const T* r = buf + Pad<T>::rpos(ny, ppitch, c, 0);
    out[j * nx + p0 + c] = r[Pad<T>::ridx(j)];
    if (dy) {
      T d = T(0);
      if (j > 0)
        d = mihy * ((j + 1 < ny ? r[Pad<T>::ridx(j + 1)] : T(0)) - r[Pad<T>::ridx(j - 1)]);
      a.out_dy[j * nx + p0 + c] = d;
    }
  }
}

// ---------------------------------------------------------------------------
// P3: inverse DST along x with epilogues
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_row_inv(Geom g, RowInvArgs<T> a, AxisTables<T> tx) {
  extern __shared__ unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  __shared__ T wsum[4];
  const int n = g.nx;
  const int R = row_block_rows(n, g.ny);
  const int ppitch = Pad<T>::pitch(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables(tx, n, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int j0 = blockIdx.x * R;
  const int fld = blockIdx.y;
  const T* in = a.in[fld];
#pragma unroll
  for (int it = 0; it < kRowMaxE; ++it) {
    const int e = threadIdx.x + it * kBlock;
    if (e >= R * n) break;
    const int r = e / n, i = e % n;
    buf[Pad<T>::rpos(n, ppitch, r, i)] = in[(j0 + r) * n + i];
  }
  __syncthreads();
  block_dst<T, kRowMaxC>(buf, g.lx, R, ppitch, tw, pre, wsum);
  guess_job(a.guess, static_cast<size_t>(g.nx) * g.ny);
  T* out = a.out[fld];
  T* out_dx = a.out_dx[fld];
  const T mihx = static_cast<T>(-0.5 / g.hx);
#pragma unroll
  for (int it = 0; it < kRowMaxE; ++it) {
    const int e = threadIdx.x + it * kBlock;
    if (e >= R * n) break;
    const int r = e / n, i = e % n;
    const int j = j0 + r;
    const T* row = buf + Pad<T>::rpos(n, ppitch, r, 0);
    const T u = j > 0 ? row[Pad<T>::ridx(i)] : T(0);
    out[j * n + i] = u;
    if (out_dx) {
      T d = T(0);
      if (i > 0 && j > 0)
        d = mihx * ((i + 1 < n ? row[Pad<T>::ridx(i + 1)] : T(0)) - row[Pad<T>::ridx(i - 1)]);
      out_dx[j * n + i] = d;
    }
  }
}

// Predictor-corrector epilogue: B_new from the inverse transform, FP64 sums
// of |B_new - B_old|^2 and |B_new|^2, B_old overwritten by B_new in place.
// The last workgroup to finish forms the relative change and decides
// convergence for the whole slice.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_row_inv_pc(Geom g, PCArgs<T> a, AxisTables<T> tx, DevCounters* ctr) {
  if (ctr->pc_done) return;
  extern __shared__ unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  __shared__ T wsum[4];
  __shared__ double red[2][kBlock / 64];
  __shared__ bool last;
  const int n = g.nx;
  const int R = row_block_rows(n, g.ny);
  const int ppitch = Pad<T>::pitch(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables(tx, n, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int j0 = blockIdx.x * R;
  const int fld = blockIdx.y;   // 0 Bx, 1 By
  const T* in = a.in + static_cast<size_t>(fld) * g.nx * g.ny;
#pragma unroll
  for (int it = 0; it < kRowMaxE; ++it) {
    const int e = threadIdx.x + it * kBlock;
    if (e >= R * n) break;
    const int r = e / n, i = e % n;
    buf[Pad<T>::rpos(n, ppitch, r, i)] = in[(j0 + r) * n + i];
  }
  __syncthreads();
  block_dst<T, kRowMaxC>(buf, g.lx, R, ppitch, tw, pre, wsum);
  T* b = fld == 0 ? a.bx : a.by;
  double dsum = 0.0, nsum = 0.0;
#pragma unroll
  for (int it = 0; it < kRowMaxE; ++it) {
    const int e = threadIdx.x + it * kBlock;
    if (e >= R * n) break;
    const int r = e / n, i = e % n;
    const int j = j0 + r;
    const T u = (j > 0) ? buf[Pad<T>::rpos(n, ppitch, r, i)] : T(0);
    const double old = static_cast<double>(b[j * n + i]);
    const double d = static_cast<double>(u) - old;
    dsum += d * d;
    nsum += static_cast<double>(u) * static_cast<double>(u);
    b[j * n + i] = u;
    T* tp = fld == 0 ? a.tape_bx : a.tape_by;
    if (tp) tp[j * n + i] = u;
  }
  // workgroup reduction
  for (int off = 32; off > 0; off >>= 1) {
    dsum += __shfl_down(dsum, off, 64);
    nsum += __shfl_down(nsum, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = dsum;
    red[1][wave] = nsum;
  }
  __syncthreads();
  const int nblk = gridDim.x * gridDim.y;
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x == 0) {
    double d = 0.0, s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      d += red[0][w];
      s += red[1][w];
    }
    a.partial[2 * bid] = d;
    a.partial[2 * bid + 1] = s;
    __threadfence();
    const unsigned int prev = atomicAdd(&ctr->blocks_arrived, 1u);
    last = (prev == static_cast<unsigned int>(nblk - 1));
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double d = 0.0, s = 0.0;
  for (int k = threadIdx.x; k < nblk; k += kBlock) {
    d += a.partial[2 * k];
    s += a.partial[2 * k + 1];
  }
  for (int off = 32; off > 0; off >>= 1) {
    d += __shfl_down(d, off, 64);
    s += __shfl_down(s, off, 64);
  }
  __syncthreads();
  if (lane == 0) {
    red[0][wave] = d;
    red[1][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double dd = 0.0, ss = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      dd += red[0][w];
      ss += red[1][w];
    }
    double res = ss > 0.0 ? sqrt(dd / ss) : (dd == 0.0 ? 0.0 : INFINITY);
    if (!isfinite(res) || !isfinite(dd) || !isfinite(ss)) ctr->nonfinite = 1u;
    ctr->pc_resid = res;
    ctr->pc_iters += 1u;
    ctr->pc_iterations += 1ull;
    ctr->blocks_arrived = 0u;
    if (a.tol > 0.0 && res < a.tol) ctr->pc_done = 1u;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Workgroups above 64 KiB of LDS (large grids, FP64) opt in explicitly; gfx950
// offers 160 KiB per workgroup.
static void allow_lds(const void* fn, size_t lds) {
  if (lds > 65536)
    QSP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(lds)));
}

template <typename T>
void launch_src_fwd_pez(const Geom& g, const SrcPEZ<T>& a, const AxisTables<T>& tx,
                        hipStream_t st) {
  const int R = row_block_rows(g.nx, g.ny);
  const size_t lds = static_cast<size_t>(R / 2) * Pad<T>::pitch(g.nx) * sizeof(T) + table_bytes<T>(g.nx);
  allow_lds(reinterpret_cast<const void*>(&k_src_fwd_pez<T>), lds);
  hipLaunchKernelGGL(k_src_fwd_pez<T>, dim3(g.ny / R, 3), dim3(kBlock), lds, st, g, a, tx);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_src_fwd_bxby(const Geom& g, const SrcBxBy<T>& a, const AxisTables<T>& tx,
                         const DevCounters* ctr, hipStream_t st) {
  const int R = row_block_rows(g.nx, g.ny);
  const size_t lds = static_cast<size_t>(R / 2) * Pad<T>::pitch(g.nx) * sizeof(T) + table_bytes<T>(g.nx);
  allow_lds(reinterpret_cast<const void*>(&k_src_fwd_bxby<T>), lds);
  hipLaunchKernelGGL(k_src_fwd_bxby<T>, dim3(g.ny / R, 2), dim3(kBlock), lds, st, g, a, tx,
                     ctr);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_col_solve(const Geom& g, const ColArgs<T>& a, int nfield, const AxisTables<T>& ty,
                      const double* lamx, const DevCounters* ctr, hipStream_t st) {
  const int W = a.w;
  if (W < 2 || (W & (W - 1)) || g.nx % W || nfield < 1 || nfield > 4)
    throw std::invalid_argument("column pass: bad strip width or field count");
  const size_t lds = static_cast<size_t>(W / 2) * Pad<T>::pitch(g.ny) * sizeof(T) + table_bytes<T>(g.ny) +
                     static_cast<size_t>(g.ny) * sizeof(double);
  allow_lds(reinterpret_cast<const void*>(&k_col_solve<T>), lds);
  hipLaunchKernelGGL(k_col_solve<T>, dim3(g.nx / W, nfield), dim3(kBlock), lds, st, g, a, ty,
                     lamx, ctr);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_row_inv(const Geom& g, const RowInvArgs<T>& a, int nfield, const AxisTables<T>& tx,
                    hipStream_t st) {
  const int R = row_block_rows(g.nx, g.ny);
  const size_t lds = static_cast<size_t>(R / 2) * Pad<T>::pitch(g.nx) * sizeof(T) + table_bytes<T>(g.nx);
  allow_lds(reinterpret_cast<const void*>(&k_row_inv<T>), lds);
  hipLaunchKernelGGL(k_row_inv<T>, dim3(g.ny / R, nfield), dim3(kBlock), lds, st, g, a, tx);
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_row_inv_pc(const Geom& g, const PCArgs<T>& a, const AxisTables<T>& tx,
                       DevCounters* ctr, hipStream_t st) {
  const int R = row_block_rows(g.nx, g.ny);
  const size_t lds = static_cast<size_t>(R / 2) * Pad<T>::pitch(g.nx) * sizeof(T) + table_bytes<T>(g.nx);
  allow_lds(reinterpret_cast<const void*>(&k_row_inv_pc<T>), lds);
  hipLaunchKernelGGL(k_row_inv_pc<T>, dim3(g.ny / R, 2), dim3(kBlock), lds, st, g, a, tx, ctr);
  QSP_LAUNCH_CHECK();
}

int pc_partial_count(const Geom& g) { return 2 * (g.ny / row_block_rows(g.nx, g.ny)); }

template <typename T>
int col_width(const Geom& g, int nfield) {
  return col_strip<T>(g.nx, g.ny, nfield);
}
template int col_width<float>(const Geom&, int);
template int col_width<double>(const Geom&, int);

#define QSP_INST(T)                                                                       \
  template void launch_src_fwd_pez<T>(const Geom&, const SrcPEZ<T>&, const AxisTables<T>&, \
                                      hipStream_t);                                        \
  template void launch_src_fwd_bxby<T>(const Geom&, const SrcBxBy<T>&,                     \
                                       const AxisTables<T>&, const DevCounters*,           \
                                       hipStream_t);                                       \
  template void launch_col_solve<T>(const Geom&, const ColArgs<T>&, int,                   \
                                    const AxisTables<T>&, const double*,                   \
                                    const DevCounters*, hipStream_t);                      \
  template void launch_row_inv<T>(const Geom&, const RowInvArgs<T>&, int,                  \
                                  const AxisTables<T>&, hipStream_t);                      \
  template void launch_row_inv_pc<T>(const Geom&, const PCArgs<T>&, const AxisTables<T>&,  \
                                     DevCounters*, hipStream_t);
QSP_INST(float)
QSP_INST(double)
#undef QSP_INST

}  // namespace qsp
