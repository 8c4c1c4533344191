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


// ---------------------------------------------------------------------------
// FP32 core for n = 256, 512, 1024 without a recurrence.  The odd outputs of
// the half-length transform above come from a prefix sum, whose FP32
// round-off grows like sqrt(n) and, through the centred differences taken of
// the solved fields, reaches ~1e-4 of Ey+Bx at 512^2-1024^2.  Here the two
// rows a, b of a pair are extended oddly to length N = 2n (z_j = a_j + i b_j,
// z_{2n-j} = -z_j, z_0 = z_n = 0) and transformed by one complex FFT of
// length N: with X = DFT_N(z), S^a_p = -Im X_p / 2 and S^b_p = Re X_p / 2.
// Every output carries plain FFT round-off.
//
// One wave per pair, N = 64 P (P = 8, 16, 32 points per lane), as a 4-step
// FFT with the index j = l + 64 m (lane l, register m) and k = k1 + P k2:
//   A   each lane: DFT_P over m in registers, times W_N^{l k1};
//   B1  DFT_64 over l split as 8 x 8 (l = la + 8 lb, k2 = c1 + 8 c2):
//       DFT_8 over lb, times W_64^{la c1};
//   B2  DFT_8 over la.
// Two transposes through the pair's LDS region (rows of 72 complex per k1:
// the transposes and the strided DFT_8 reads touch every bank once per two
// rows), no workgroup barrier.
// ---------------------------------------------------------------------------
constexpr int kCorePitch = 72;   // complex entries per k1 row of the transposes

// Row layout in LDS around the FP32 core (gfx950 serves LDS as 32 banks of 4
// bytes, half a wave at a time): 4 padding words after every 32, row b of a
// pair at an offset = 4 (mod 32), pairs 8 (mod 32) apart (at 1024 points: 8
// and 16).  Then the core's last-stage writes (k = kb + P c1 + const over
// the lanes kb < 4, c1 < 8 of a half-wave) land on 32 distinct banks, and
// so do the column pass's strip accesses (8 columns = 4 pairs x 2 rows, 4
// consecutive rows each; at 1024 points 4 columns, 8 rows each); runs of 32
// consecutive entries (row passes, the core's first stage) stay contiguous.
struct CoreLay {
  __host__ __device__ static constexpr int ridx(int i) { return i + 4 * (i >> 5); }
  // offset of row b in the pair (named as in Pad): = 4 (mod 32), or = 8 at
  // 1024 points, whose column strips are 4 columns (2 pairs) wide
  __host__ __device__ static constexpr int rlen(int n) {
    return ((ridx(n) + 31) & ~31) + (n >= 1024 ? 8 : 4);
  }
  __host__ __device__ static constexpr int rpos(int n, int pitch, int r, int i) {
    return (r >> 1) * pitch + (r & 1) * rlen(n) + ridx(i);
  }
};

// W_32^k = e^{-2 pi i k / 32} for k >= 0 (from cos(2 pi k / 32), k = 0..8;
// W_32^{k+16} = -W_32^k).  Called with compile-time k only.
__device__ __forceinline__ Cplx<float> w32(int k) {
  constexpr double c32[9] = {1.0,
                             0.98078528040323044913,
                             0.92387953251128675613,
                             0.83146961230254523708,
                             0.70710678118654752440,
                             0.55557023301960222474,
                             0.38268343236508977173,
                             0.19509032201612826785,
                             0.0};
  const double sg = (k & 16) ? -1.0 : 1.0;
  k &= 15;
  const double c = k <= 8 ? c32[k] : -c32[16 - k];
  const double s = k <= 8 ? c32[8 - k] : c32[k - 8];
  return {static_cast<float>(sg * c), static_cast<float>(-sg * s)};
}

// In-register forward DFT of length P = R1 * 8 (R1 = 1, 2, 4), in place with
// j = j0 + 8 j1 and k = k0 + R1 k1: DFT_R1 over j1, twiddles W_P^{j0 k0},
// DFT_8 over j0.  X_k ends at position dft_pos<P>(k) = 8 k0 + k1.
template <int P>
__host__ __device__ constexpr int dft_pos(int k) {
  return 8 * (k % (P / 8)) + k / (P / 8);
}

template <int P>
__device__ __forceinline__ void dft_reg(Cplx<float>* v) {
  constexpr int R1 = P / 8;
  if constexpr (R1 == 2) {
#pragma unroll
    for (int j0 = 0; j0 < 8; ++j0) {
      const Cplx<float> a = v[j0], b = v[j0 + 8];
      v[j0] = cadd(a, b);
      v[j0 + 8] = csub(a, b);
    }
  } else if constexpr (R1 == 4) {
#pragma unroll
    for (int j0 = 0; j0 < 8; ++j0) dft4(v[j0], v[j0 + 8], v[j0 + 16], v[j0 + 24]);
  }
  if constexpr (R1 > 1) {
#pragma unroll
    for (int k0 = 1; k0 < R1; ++k0)
#pragma unroll
      for (int j0 = 1; j0 < 8; ++j0) v[8 * k0 + j0] = cmul(v[8 * k0 + j0], w32(j0 * k0 * (32 / P)));
  }
#pragma unroll
  for (int k0 = 0; k0 < R1; ++k0) dft8(v + 8 * k0);
}

// DST-I of one pair (rows a at g, b at g + rlen(n), entry 0 = 0) by one
// wave, in place; twa[k1 * 64 + l] = W_N^{l k1} (global memory), w64[la * 9
// + c1] = W_64^{la c1} (LDS).  The pair's region holds P rows of kCorePitch
// complex.
// Output scaling of the core: none (plain transform).  The cores call
// epi(q, oa, ob) for their q-th output slot of the lane.
struct NoScale {
  __device__ void operator()(int, float&, float&) const {}
};

// Output scaling of the core in the column pass: S_k of the pair's columns
// p_a, p_b divided by (lambda_x(p) + lambda_y(k) - shift) nx ny / 4, the
// eigenvalue of the shifted Laplacian times the two transforms'
// normalisation; column p = 0 (a boundary node line) is zero.  ry holds
// (lambda_y(k) - shift) nx ny / 4 for the lane's NK output slots k (see
// core_out_k), xa / xb lambda_x(p) nx ny / 4.
template <int NK>
struct EigenScale {
  float ry[NK];
  float xa, xb;
  bool za;
  __device__ void operator()(int q, float& oa, float& ob) const {
    const float ra = __builtin_amdgcn_rcpf(xa + ry[q]);
    const float rb = __builtin_amdgcn_rcpf(xb + ry[q]);
    oa = za ? 0.f : oa * ra;
    ob *= rb;
  }
};

// Output slots of a lane: the one-wave core (P points per lane, lane l)
// writes k = (l >> 3) + 8 t + P (l & 7) + 8 P c2 in slot q = 4 t + c2; the
// two-wave core (P points per lane, lane L of 128) k = k1 + P c1 + 8 P q with
// k1 = (L >> 6) P / 2 + ((L & 63) >> 3), c1 = L & 7 (lanes whose k1 falls
// outside their wave's rows write nothing; their k is wrapped into [0, n)).
template <int P>
__device__ __forceinline__ int core_out_k(int l, int q) {
  return (l >> 3) + 8 * (q >> 2) + P * (l & 7) + 8 * P * (q & 3);
}
template <int P>
__device__ __forceinline__ int core2_out_k(int L, int q) {
  return ((L >> 6) * (P / 2) + ((L & 63) >> 3) + P * (L & 7) + 8 * P * q) & (64 * P - 1);
}

template <int P, typename Epi = NoScale>
__device__ __forceinline__ void wave_dst_core(float* g, const Cplx<float>* __restrict__ twa,
                                              const Cplx<float>* __restrict__ w64,
                                              const Epi& epi = Epi{}) {
  using Pd = CoreLay;
  constexpr int n = 32 * P;
  constexpr int NB = P / 8;
  const int l = threadIdx.x & 63;
  float* ra = g;
  float* rb = g + Pd::rlen(n);
  Cplx<float>* s = reinterpret_cast<Cplx<float>*>(g);
  // A: z_{l + 64 m}; m >= P/2 from the mirror 2n - j = 64 (P - m) - l
  Cplx<float> v[P];
#pragma unroll
  for (int m = 0; m < P / 2; ++m) {
    const int j = Pd::ridx(l + 64 * m);
    v[m] = {ra[j], rb[j]};
  }
#pragma unroll
  for (int m = P / 2; m < P; ++m) {
    const int jm = 64 * (P - m) - l;          // in [1, n], n only for l = 0, m = P/2
    const int j = Pd::ridx(jm < n ? jm : 0);
    const float fa = ra[j], fb = rb[j];
    v[m] = {jm < n ? -fa : 0.f, jm < n ? -fb : 0.f};
  }
  wave_sync();
  dft_reg<P>(v);
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) {
    const Cplx<float> y = v[dft_pos<P>(k1)];
    s[k1 * kCorePitch + l] = k1 ? cmul(y, twa[k1 * 64 + l]) : y;
  }
  wave_sync();
  // B1: combos (k1, la) = (l >> 3 + 8 t, l & 7)
  const int la = l & 7, kb = l >> 3;
  Cplx<float> u[NB][8];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const Cplx<float>* r = s + (kb + 8 * t) * kCorePitch + la;
#pragma unroll
    for (int lb = 0; lb < 8; ++lb) u[t][lb] = r[8 * lb];
  }
  Cplx<float> wl[8];
  wl[0] = {1.f, 0.f};
#pragma unroll
  for (int c1 = 1; c1 < 8; ++c1) wl[c1] = w64[la * 9 + c1];
  wave_sync();
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    dft8(u[t]);
    Cplx<float>* r = s + (kb + 8 * t) * kCorePitch + la * 9;
    r[0] = u[t][0];
#pragma unroll
    for (int c1 = 1; c1 < 8; ++c1) r[c1] = cmul(u[t][c1], wl[c1]);
  }
  wave_sync();
  // B2: combos (k1, c1) = (l >> 3 + 8 t, l & 7); DFT_8 over la
  const int c1 = l & 7;
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const Cplx<float>* r = s + (kb + 8 * t) * kCorePitch + c1;
#pragma unroll
    for (int a = 0; a < 8; ++a) u[t][a] = r[a * 9];
  }
  wave_sync();
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    dft8(u[t]);
    const int k0 = kb + 8 * t + P * c1;       // k = k0 + 8 P c2, < n for c2 < 4
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      const int k = k0 + 8 * P * c2;
      const int j = Pd::ridx(k);
      float oa = -0.5f * u[t][c2].im, ob = 0.5f * u[t][c2].re;
      epi(4 * t + c2, oa, ob);
      ra[j] = k ? oa : 0.f;
      rb[j] = k ? ob : 0.f;
    }
  }
  wave_sync();
}

// ---------------------------------------------------------------------------
// Two-wave FP32 core for rows of n = 64 P points (used with P = 16, n = 1024):
// the pair's 128 lanes share the N = 128 P-point FFT, P points per lane, so
// that twice as many waves (two per SIMD on a full grid) hide each other's
// latencies:
//   A   lane L: DFT_P over m of z_{L + 128 m}, times W_N^{L k1} (k = k1 +
//       P k2), into row k1 of the transpose region; one workgroup barrier;
//   B1  DFT_128 over L split as 16 x 8 (L = la + 16 lb, k2 = c1 + 8 c2):
//       DFT_8 over lb, times W_128^{la c1}; wave w of the pair owns rows
//       k1 = w P/2 .. (w + 1) P/2 - 1 from here on (no more barriers);
//   B2  DFT_16 over la (4 P of a wave's 64 lanes), outputs k = k1 + P c1 +
//       8 P c2 for c2 < 8.
// The transposes use a region of their own after the rows (rows of 152
// complex: the strided reads and writes of B1 and B2 meet every bank once
// per 16 lanes), so the first stage reads its rows without a barrier before
// its writes.  Every thread of the workgroup must call it (its barrier);
// the caller synchronises the workgroup before the rows are read again.
// ---------------------------------------------------------------------------
constexpr int kCore2Pitch = 152;   // complex entries per k1 row of the transposes

__host__ __device__ constexpr int core2_soff(int n) {   // floats before the transposes
  return (CoreLay::rlen(n) + CoreLay::ridx(n) + 31) & ~31;
}

template <int P, typename Epi = NoScale>
__device__ __forceinline__ void pair2_dst_core(float* g, int L, const Cplx<float>* __restrict__ twa,
                                               const Cplx<float>* __restrict__ w128,
                                               const Epi& epi = Epi{}) {
  using Pd = CoreLay;
  constexpr int n = 64 * P;
  constexpr int HR = P / 2;   // transpose rows per wave
  float* ra = g;
  float* rb = g + Pd::rlen(n);
  Cplx<float>* s = reinterpret_cast<Cplx<float>*>(g + core2_soff(n));
  // A: z_{L + 128 m}; m >= P/2 from the mirror 2n - j = 128 (P - m) - L
  Cplx<float> v[P];
#pragma unroll
  for (int m = 0; m < P / 2; ++m) {
    const int j = Pd::ridx(L + 128 * m);
    v[m] = {ra[j], rb[j]};
  }
#pragma unroll
  for (int m = P / 2; m < P; ++m) {
    const int jm = 128 * (P - m) - L;         // in [1, n], n only for L = 0, m = P/2
    const int j = Pd::ridx(jm < n ? jm : 0);
    const float fa = ra[j], fb = rb[j];
    v[m] = {jm < n ? -fa : 0.f, jm < n ? -fb : 0.f};
  }
  dft_reg<P>(v);
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) {
    const Cplx<float> y = v[dft_pos<P>(k1)];
    s[k1 * kCore2Pitch + L] = k1 ? cmul(y, twa[k1 * 128 + L]) : y;
  }
  __syncthreads();
  // B1: lane (la, kb) of wave w handles rows k1 = w HR + kb + 4 t
  const int l6 = L & 63, w = L >> 6;
  const int la = l6 & 15, kb = l6 >> 4;
  constexpr int NT = HR / 4;
  Cplx<float> u[NT][8];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const Cplx<float>* r = s + (w * HR + kb + 4 * t) * kCore2Pitch + la;
#pragma unroll
    for (int lb = 0; lb < 8; ++lb) u[t][lb] = r[16 * lb];
  }
  Cplx<float> wl[8];
  wl[0] = {1.f, 0.f};
#pragma unroll
  for (int c1 = 1; c1 < 8; ++c1) wl[c1] = w128[la * 9 + c1];
  wave_sync();
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    dft8(u[t]);
    Cplx<float>* r = s + (w * HR + kb + 4 * t) * kCore2Pitch + la * 9;
    r[0] = u[t][0];
#pragma unroll
    for (int c1 = 1; c1 < 8; ++c1) r[c1] = cmul(u[t][c1], wl[c1]);
  }
  wave_sync();
  // B2: lane (k1, c1) = (w HR + l6 >> 3, l6 & 7) for l6 < 8 HR; DFT_16 over la
  if ((l6 >> 3) < HR) {
    const int k1 = w * HR + (l6 >> 3), c1 = l6 & 7;
    Cplx<float> x[16];
    const Cplx<float>* r = s + k1 * kCore2Pitch + c1;
#pragma unroll
    for (int a = 0; a < 16; ++a) x[a] = r[9 * a];
    dft_reg<16>(x);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const Cplx<float> y = x[dft_pos<16>(q)];
      const int k = k1 + P * c1 + 8 * P * q;
      const int j = Pd::ridx(k);
      float oa = -0.5f * y.im, ob = 0.5f * y.re;
      epi(q, oa, ob);
      ra[j] = k ? oa : 0.f;
      rb[j] = k ? ob : 0.f;
    }
  }
}

// Floats per row pair in LDS: the two padded rows, or for the FP32 core the
// P rows of its transposes (which the one-wave core lays over the rows), or
// for the two-wave core the rows followed by its transposes.
template <typename T>
__host__ __device__ inline int pair_pitch(int n) {
  if (fast_core(sizeof(T), n) && core_lanes(sizeof(T), n) == 128)   // rows, transposes; = 16 (mod 32)
    return core2_soff(n) + (n / 64) * kCore2Pitch * 2 + 16;
  if (fast_core(sizeof(T), n)) return (n / 32) * kCorePitch * 2 + 8;   // = 8 (mod 32)
  return Pad<T>::pitch(n);
}

// The LDS row layout of a pass over rows of 2^LOGN values.
template <typename T, int LOGN>
using RowLay = std::conditional_t<fast_core(sizeof(T), 1 << LOGN), CoreLay, Pad<T>>;

// Type-I sine transform of nrow rows (nrow even) of length n = 2^logn held
// in LDS; pair f = rows (2f, 2f+1) occupies buf[f*ppitch ..) (row 2f first,
// ppitch = pair_pitch(n)).  Entry 0 of every input row must be 0; on output
// entry p holds S_p (entry 0 = 0).  FP32 rows of 256-1024 go to the
// recurrence-free core, one pair per wave; otherwise groups of max(1, 512/n)
// pairs are handed to the workgroup's waves in turn.  Ends with a workgroup
// barrier.
template <typename T, int LOGN>
__device__ __forceinline__ void block_dst(T* buf, int logn, int nrow, int ppitch,
                                          const Cplx<T>* __restrict__ tw,
                                          const T* __restrict__ pre) {
  constexpr int n = 1 << LOGN;
  (void)logn;
  const int npair = nrow >> 1;
  const int wave = threadIdx.x >> 6;
  if constexpr (fast_core(sizeof(T), n)) {
    // tw: W_N^{l k1} by [k1][lane]; pre: the W_64 (W_128) table (complex)
    const Cplx<float>* wt = reinterpret_cast<const Cplx<float>*>(pre);
    if constexpr (core_lanes(sizeof(T), n) == 128) {
      // two waves per pair, every thread (the launchers give 4 rows: 2 pairs)
      const int pr = threadIdx.x >> 7;
      pair2_dst_core<n / 64>(buf + static_cast<size_t>(pr) * ppitch, threadIdx.x & 127, tw, wt);
    } else {
      // one pair per wave (the launchers keep nrow <= 2 * waves): no loop,
      // whose invariant hoisting would keep the core's per-lane addresses live
      if (wave < npair) wave_dst_core<n / 32>(buf + static_cast<size_t>(wave) * ppitch, tw, wt);
    }
  } else {
    constexpr int per = n >= 512 ? 1 : 512 / n;
    constexpr int E = n <= 512 ? 8 : n / 64;
    // at most one group per wave (the launchers keep nrow <= 2 * per * waves)
    const int ngroup = (npair + per - 1) / per;
    if (wave < ngroup) {
      const int npg = min(per, npair - wave * per);
      wave_dst<T, E, LOGN>(buf + static_cast<size_t>(wave) * per * ppitch, npg, ppitch, tw, pre);
    }
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

// Bytes of the per-axis tables a transform pass stages in LDS: twiddles and
// pre-twiddles of the half-length transform; for the one-wave FP32 core the
// W_64 table (72 complex; its W_N^{l k1} table is read from global memory);
// for the two-wave core both (2n + 144 complex), so that its transforms
// issue no global loads (a wait on a load also waits on earlier stores).
template <typename T>
__host__ __device__ inline size_t table_bytes(int n) {
  if (fast_core(sizeof(T), n) && core_lanes(sizeof(T), n) == 128)   // W_N and W_128 tables
    return static_cast<size_t>(2 * n + 144) * sizeof(Cplx<T>);
  if (fast_core(sizeof(T), n)) return static_cast<size_t>(core_lanes(sizeof(T), n) / 8 * 9) * sizeof(Cplx<T>);
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

// Eigenvalue bytes the column pass stages after the tables: the strip's W
// x eigenvalues, and the n y eigenvalues except with the FP32 core (which
// reads them from global memory so that two workgroups fit a CU at 1024).
template <typename T>
__host__ __device__ inline size_t lam_bytes(int n, int w) {
  return static_cast<size_t>((fast_core(sizeof(T), n) ? 0 : n) + w) * sizeof(double);
}

template <typename T>
inline size_t pass_lds(int rows, int n) {
  return static_cast<size_t>(rows / 2) * pair_pitch<T>(n) * sizeof(T) + table_bytes<T>(n) +
         lam_bytes<T>(n, rows);
}

// columns per column-pass workgroup (even, at most nx, within 80 KiB of LDS).
// One busy wave (one column pair) per workgroup up to 512 rows (FP32) or
// 256 rows (FP64); beyond, two, whose four-column strips halve the strided
// row segments each workgroup reads (measured from HIP graphs: 8 % off a
// 1024^2 time step in FP32, 2 % off the 512^2 box in FP64).
// The FP32 core at 1024 rows: two pairs of two waves (four-column strips),
// two workgroups per CU.
template <typename T>
inline int col_strip(int nx, int ny, int nfield) {
  (void)nfield;
  if (core_lanes(sizeof(T), ny) == 128) return 4;   // two-wave core: two pairs per workgroup
  const bool core = fast_core(sizeof(T), ny);
  const int per = ny >= 512 || core ? 1 : 512 / ny;
  const int waves = core ? (ny >= 1024 ? 4 : 1) : (ny >= (sizeof(T) == 8 ? 512 : 1024) ? 2 : 1);
  int w = 2 * per * pass_waves("QSP_COL_WAVES", waves);
  if (const char* e = std::getenv("QSP_COL_W")) {   // tuning override
    const int v = std::atoi(e);
    if (v >= 2 && v <= 64 && (v & (v - 1)) == 0) w = v;
  }
  if (w > nx) w = nx;
  if (w > 2 * per * (kBlock / 64)) w = 2 * per * (kBlock / 64);   // one pair group per wave
  const size_t cap = 81920;   // two workgroups per CU
  while (w > 2 && pass_lds<T>(w, ny) > cap) w >>= 1;
  return w;
}

// Copies an axis' transform tables into LDS right after the workgroup's data
// region, so the FFT stages never wait on global memory.  Every load of a
// thread is issued before its first LDS store (one memory latency, not one
// per loop trip).
template <typename T, int LOGN>
__device__ inline void stage_tables(const AxisTables<T>& t, unsigned char* base,
                                    const Cplx<T>*& tw, const T*& pre) {
  constexpr int n = 1 << LOGN;
  Cplx<T>* stw = reinterpret_cast<Cplx<T>*>(base);
  if constexpr (fast_core(sizeof(T), n)) {
    // the W_N^{l k1} table (2n entries by [k1][lane]) stays in global
    // memory, where each wave reads it coalesced (L1/L2 resident); the 72
    // (144) entries of W_64 (W_128) go to LDS
    Cplx<T>* sw = stw;
    const Cplx<T>* gw = reinterpret_cast<const Cplx<T>*>(t.pre);
    if constexpr (core_lanes(sizeof(T), n) == 128) {
      // W_N^{L k1} (2n entries) then W_128 (144) in LDS
      constexpr int NT = 2 * n / kBlock;
      Cplx<T> v[NT];
#pragma unroll
      for (int u = 0; u < NT; ++u) v[u] = t.tw[threadIdx.x + u * kBlock];
      const Cplx<T> wv = threadIdx.x < 144 ? gw[threadIdx.x] : Cplx<T>{T(0), T(0)};
#pragma unroll
      for (int u = 0; u < NT; ++u) sw[threadIdx.x + u * kBlock] = v[u];
      if (threadIdx.x < 144) sw[2 * n + threadIdx.x] = wv;
      tw = sw;
      pre = reinterpret_cast<const T*>(sw + 2 * n);
    } else {
      if (threadIdx.x < core_lanes(sizeof(T), n) / 8 * 9) sw[threadIdx.x] = gw[threadIdx.x];
      tw = t.tw;
      pre = reinterpret_cast<const T*>(sw);
    }
  } else {
    T* spre = reinterpret_cast<T*>(base + n * sizeof(Cplx<T>));
    if constexpr (n % kBlock == 0) {
      constexpr int NT = n / kBlock;
      Cplx<T> v[NT];
      T q[NT];
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        v[u] = t.tw[threadIdx.x + u * kBlock];
        q[u] = t.pre[threadIdx.x + u * kBlock];
      }
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        stw[threadIdx.x + u * kBlock] = v[u];
        spre[threadIdx.x + u * kBlock] = q[u];
      }
    } else if (threadIdx.x < n) {   // n < kBlock
      stw[threadIdx.x] = t.tw[threadIdx.x];
      spre[threadIdx.x] = t.pre[threadIdx.x];
    }
    tw = stw;
    pre = spre;
  }
}

// dst[i] = src[i] for i < N, all of a thread's loads before its stores
template <int N>
__device__ inline void stage_doubles(double* dst, const double* __restrict__ src) {
  if constexpr (N % kBlock == 0) {
    constexpr int NT = N / kBlock;
    double v[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) v[u] = src[threadIdx.x + u * kBlock];
#pragma unroll
    for (int u = 0; u < NT; ++u) dst[threadIdx.x + u * kBlock] = v[u];
  } else if (threadIdx.x < N) {   // N < kBlock
    dst[threadIdx.x] = src[threadIdx.x];
  }
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
  // rounds of 8 elements per thread with all their loads issued first
  constexpr int U = 8;
  for (size_t i0 = bid * blockDim.x + threadIdx.x; i0 < n; i0 += U * stride) {
    T vx[U], vy[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = i0 + u * stride;
      const size_t c = i < n ? i : 0;   // clamped: every load in bounds
      vx[u] = T(2) * q.bx1[c] - q.bx2[c];
      vy[u] = T(2) * q.by1[c] - q.by2[c];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = i0 + u * stride;
      if (i < n) {
        q.bx[i] = vx[u];
        q.by[i] = vy[u];
        if (q.tape_bx) {
          q.tape_bx[i] = vx[u];
          q.tape_by[i] = vy[u];
        }
      }
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
// The FP32 core holds P = 2n/64 complex points per lane (one pair per wave,
// up to ~140 VGPRs at 1024 points): two workgroups per CU at 1024, four
// below.
constexpr int dst_blocks_per_cu(int logn, int tsize) {
  if (fast_core(tsize, 1 << logn)) return logn >= 10 ? 2 : 4;
  const int u = (logn <= 9 ? 8 : (1 << logn) / 64) * tsize / 4;
  return u <= 8 ? 4 : (u <= 16 ? 2 : 1);
}

// The column pass with the FP32 core keeps its eigenvalue divisors and a
// strip load in flight beside the core's registers: two workgroups per CU
// (its grids hold at most two per CU at 512 and 1024 rows).
constexpr int col_blocks_per_cu(int logn, int tsize) {
  if (fast_core(tsize, 1 << logn)) return 2;
  const int u = (logn <= 9 ? 8 : (1 << logn) / 64) * tsize / 4;
  return u <= 8 ? 4 : (u <= 16 ? 2 : 1);
}

// Calls f(e) for the workgroup's elements e = threadIdx.x + it*kBlock,
// e < total.  The whole multiples of kBlock run as unrolled straight-line
// chunks of up to CH (8, 16 or 32), so with a branch-free f the global loads
// of a chunk are in flight together instead of one load latency per element
// (plain copies take 32, source assembly with several loads per element 8).
template <int CH, typename F>
__device__ __forceinline__ void elem_chunk(int& it, F& f) {
#pragma unroll
  for (int u = 0; u < CH; ++u) f(static_cast<int>(threadIdx.x) + (it + u) * kBlock);
  it += CH;
}

template <int CH = 8, typename F>
__device__ __forceinline__ void for_elems(int total, F&& f) {
  const int nit = total / kBlock;   // uniform across the workgroup
  int it = 0;
  if constexpr (CH >= 32)
    while (it + 32 <= nit) elem_chunk<32>(it, f);
  if constexpr (CH >= 16)
    while (it + 16 <= nit) elem_chunk<16>(it, f);
  while (it + 8 <= nit) elem_chunk<8>(it, f);
  if (nit & 4) elem_chunk<4>(it, f);
  if (nit & 2) elem_chunk<2>(it, f);
  if (nit & 1) elem_chunk<1>(it, f);
  for (int e = nit * kBlock + static_cast<int>(threadIdx.x); e < total; e += kBlock) f(e);
}



// Calls f(e) for e = t + u kBlock, u = 0 .. TOTAL / kBlock - 1 (TOTAL a
// multiple of kBlock known at compile time), fully unrolled: with the row
// length a compile-time power of two, the row and column of e and their LDS
// offsets fold to per-thread constants plus immediates.
template <int TOTAL, typename F>
__device__ __forceinline__ void for_elems_ct(F&& f) {
  static_assert(TOTAL % kBlock == 0, "whole multiples of the workgroup");
  const int t = static_cast<int>(threadIdx.x) & (kBlock - 1);
#pragma unroll
  for (int u = 0; u < TOTAL / kBlock; ++u) f(t + u * kBlock);
}

// The elements of a block of rows of n = 2^LOGN: RC rows when RC > 0 (a
// compile-time row count), else R rows in chunks of CH (see for_elems).
template <int RC, int LOGN, int CH = 8, typename F>
__device__ __forceinline__ void for_row_elems(int R, F&& f) {
  if constexpr (RC > 0)
    for_elems_ct<(RC << LOGN)>(f);
  else
    for_elems<CH>(R << LOGN, f);
}

// Element e of a block of 4 rows in the strip order (Geom::strip): e = 16 s
// + 4 r + c is row r, column 4 s + c, stored at offset (s ny + j0 + r) 4 + c
// of the plane, so 16 consecutive elements are one 64-byte block.
__device__ __forceinline__ void strip_elem(int e, int& r, int& i) {
  const int w = e & 15;
  r = w >> 2;
  i = ((e >> 4) << 2) | (w & 3);
}
__device__ __forceinline__ size_t strip_off(int e, int j0, int ny) {
  return static_cast<size_t>(e >> 4) * (static_cast<size_t>(ny) << 2) + (static_cast<size_t>(j0) << 2) +
         (e & 15);
}

// The R rows j0.. of a row block between LDS and an intermediate plane of a
// solve: row-major, or in the strip order (Geom::strip, R = 4).
template <typename T, int RC, int LOGN, int CH = 8>
__device__ __forceinline__ void rows_to_plane(const Geom& g, int R, int j0, const T* buf, int ppitch,
                                              T* __restrict__ out) {
  constexpr int n = 1 << LOGN;
  if (g.strip) {
    for_row_elems<RC, LOGN, CH>(R, [&](int e) {
      int r, i;
      strip_elem(e, r, i);
      out[strip_off(e, j0, g.ny)] = buf[RowLay<T, LOGN>::rpos(n, ppitch, r, i)];
    });
  } else {
    for_row_elems<RC, LOGN, CH>(R, [&](int e) {
      const int r = e >> LOGN, i = e & (n - 1);
      out[(j0 + r) * n + i] = buf[RowLay<T, LOGN>::rpos(n, ppitch, r, i)];
    });
  }
}
template <typename T, int RC, int LOGN, int CH = 32>
__device__ __forceinline__ void plane_to_rows(const Geom& g, int R, int j0, const T* __restrict__ in,
                                              T* buf, int ppitch) {
  constexpr int n = 1 << LOGN;
  if (g.strip) {
    for_row_elems<RC, LOGN, CH>(R, [&](int e) {
      int r, i;
      strip_elem(e, r, i);
      buf[RowLay<T, LOGN>::rpos(n, ppitch, r, i)] = in[strip_off(e, j0, g.ny)];
    });
  } else {
    for_row_elems<RC, LOGN, CH>(R, [&](int e) {
      const int r = e >> LOGN, i = e & (n - 1);
      buf[RowLay<T, LOGN>::rpos(n, ppitch, r, i)] = in[(j0 + r) * n + i];
    });
  }
}

// Runs f(std::integral_constant<int, RC>) with RC = R (2, 4 or 8; 4 for
// the two-wave core) for row passes of the FP32 core, RC = 0 (rows at run
// time) otherwise.
template <typename T, int LOGN, typename F>
void with_rows(int R, F&& f) {
  if constexpr (core_lanes(sizeof(T), 1 << LOGN) == 128) {   // the two-wave core: 4 rows only
    if (R != 4) throw std::invalid_argument("row pass: the two-wave core takes 4 rows");
    f(std::integral_constant<int, 4>{});
  } else if constexpr (fast_core(sizeof(T), 1 << LOGN)) {
    switch (R) {
      case 2: f(std::integral_constant<int, 2>{}); break;
      case 4: f(std::integral_constant<int, 4>{}); break;
      case 8: f(std::integral_constant<int, 8>{}); break;
      default: throw std::invalid_argument("row pass: rows per workgroup must be 2, 4 or 8");
    }
  } else {
    f(std::integral_constant<int, 0>{});
  }
}

// Source assembly (FP64) + forward DST along x of row block bxi of field
// fld (0 Bx, 1 By) of the Bx/By predictor-corrector.
template <typename T, int LOGN, int RC>
__device__ __forceinline__ void src_bxby_block(const Geom& g, const SrcBxBy<T>& a,
                                               const AxisTables<T>& tx, int bxi, int fld,
                                               unsigned char* smem_raw) {
  __syncthreads();   // the workgroup's previous use of LDS is complete
  T* buf = reinterpret_cast<T*>(smem_raw);
  constexpr int n = 1 << LOGN;   // = nx
  const int R = RC > 0 ? RC : g.rr;
  const int ppitch = pair_pitch<T>(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables<T, LOGN>(tx, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int j0 = bxi * R;
  const double ihx = 0.5 / g.hx, ihy = 0.5 / g.hy;
  const double idz = 0.5 / a.dzeta;
  const double amp = a.beam_amp;
  for_row_elems<RC, LOGN>(R, [&](int e) {
    const int r = e >> LOGN, i = e & (n - 1);
    const int j = j0 + r;
    const int o = j * n + i;
    double s;
    if (fld == 0) {
      // -d_y Jz + (Jy_{k-1} - Jy_{k+1}) / (2 dzeta) - shift * Bx_old
      const int js = j > 0 ? j - 1 : 0;
      const double zs = a.jz[js * n + i], zn = a.jz[(j + 1 < g.ny ? j + 1 : j) * n + i];
      const double yp = a.jy_prev[o], yt = a.jy_next[o] + a.sy_next[o];
      const double bo = static_cast<double>(a.bx[o]);
      const double gx = a.bgx[i], gs = a.bgy[js], gn = a.bgy[j + 1];
      const double jz_s = zs - amp * gx * gs;
      const double jz_n = j + 1 < g.ny ? zn - amp * gx * gn : 0.0;
      s = -(jz_n - jz_s) * ihy + (yp - yt) * idz - a.shift * bo;
    } else {
      // d_x Jz - (Jx_{k-1} - Jx_{k+1}) / (2 dzeta) - shift * By_old
      const int iw = i > 0 ? i - 1 : 0;
      const double zw = a.jz[j * n + iw], ze = a.jz[j * n + (i + 1 < n ? i + 1 : i)];
      const double xp = a.jx_prev[o], xt = a.jx_next[o] + a.sx_next[o];
      const double bo = static_cast<double>(a.by[o]);
      const double gy = a.bgy[j], gw = a.bgx[iw], ge = a.bgx[i + 1];
      const double jz_w = zw - amp * gw * gy;
      const double jz_e = i + 1 < n ? ze - amp * ge * gy : 0.0;
      s = (jz_e - jz_w) * ihx - (xp - xt) * idz - a.shift * bo;
    }
    buf[RowLay<T, LOGN>::rpos(n, ppitch, r, i)] = static_cast<T>((i > 0 && j > 0) ? s : 0.0);
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  rows_to_plane<T, RC, LOGN>(g, R, j0, buf, ppitch, a.out + static_cast<size_t>(fld) * g.nx * g.ny);
}

// Calls f(it) for it = 0 .. NIT-1 in unrolled chunks of up to 32 (NIT a
// compile-time count), so that element addresses are affine in it.
template <int NIT, typename F>
__device__ __forceinline__ void for_iters(F&& f) {
#pragma unroll
  for (int i0 = 0; i0 < NIT; i0 += 32) {
#pragma unroll
    for (int u = 0; u < (NIT - i0 < 32 ? NIT - i0 : 32); ++u) f(i0 + u);
  }
}

// Column pass with the FP32 core (n = ny = 256..1024, W = 2, 4 or 8
// columns; at 1024 the two-wave core on 4 columns): strip load, forward
// core whose output stage divides by the eigenvalues, inverse core, store.  Thread t handles column c = t mod W and
// rows j = t / W + it (256 / W); the row step is a multiple of 32, so the
// padded LDS index ridx(j) = j + 4 (j / 32) is affine in it as well.
template <int LOGN, int W>
__device__ __forceinline__ void col_block_core(const Geom& g, const ColArgs<float>& a,
                                               const AxisTables<float>& ty,
                                               const double* __restrict__ lamx, int strip, int fld,
                                               unsigned char* smem_raw) {
  using Pd = CoreLay;
  constexpr int n = 1 << LOGN;
  constexpr bool two = core_lanes(4, n) == 128;   // two waves per pair (W = 4)
  constexpr int P = n / 32, NB = P / 8;
  constexpr int NK = two ? 8 : 4 * NB;            // output slots per lane
  constexpr int LW = W == 2 ? 1 : (W == 4 ? 2 : 3);
  constexpr int JS = kBlock / W;              // row step of a thread
  constexpr int NIT = n / JS;                 // rows per thread
  constexpr int LS = Pd::ridx(JS);            // LDS step of ridx
  static_assert(JS % 32 == 0, "row step must keep the LDS padding affine");
  static_assert(!two || W == 4, "the two-wave core takes four-column strips");
  __syncthreads();   // the workgroup's previous use of LDS is complete
  float* buf = reinterpret_cast<float*>(smem_raw);
  const int nx = g.nx;
  const int ppitch = pair_pitch<float>(n);
  const int p0 = strip * W;
  const int tid = static_cast<int>(threadIdx.x);
  const int pr = two ? tid >> 7 : tid >> 6;     // the thread's pair
  const int l = two ? tid & 127 : tid & 63;     // its lane in the pair
  const bool busy = two || pr < W / 2;
  const Cplx<float>* tw;   // W_N^{l k1}: LDS for the two-wave core, else global
  const float* wpre;
  stage_tables<float, LOGN>(ty, smem_raw + static_cast<size_t>(W / 2) * ppitch * sizeof(float), tw, wpre);
  const Cplx<float>* wt = reinterpret_cast<const Cplx<float>*>(wpre);
  // the y eigenvalues of the lane's core outputs, fetched under the strip load
  double ly[NK];
  double lxa = 0.0, lxb = 0.0;
  if (busy) {
#pragma unroll
    for (int q = 0; q < NK; ++q) ly[q] = ty.lam[two ? core2_out_k<n / 64>(l, q) : core_out_k<P>(l, q)];
    lxa = lamx[p0 + 2 * pr];
    lxb = lamx[p0 + 2 * pr + 1];
  }
  const size_t plane = static_cast<size_t>(nx) * n;
  const int c = tid & (W - 1), j0 = tid >> LW;
  const int lcol = (c >> 1) * ppitch + (c & 1) * Pd::rlen(n) + Pd::ridx(j0);
  // strip-ordered planes (Geom::strip): the strip is one contiguous block of
  // n rows x 4 columns, read and written as one float4 per row
  const bool cont = two && g.strip != 0;
  constexpr int NQ = n / kBlock;
  const int rl = Pd::rlen(n);
  if (cont) {
    const float4* src = reinterpret_cast<const float4*>(a.in + fld * plane + static_cast<size_t>(strip) * 4 * n);
    float4 v[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) v[u] = src[tid + u * kBlock];
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      float* d = buf + Pd::ridx(tid) + Pd::ridx(u * kBlock);
      d[0] = v[u].x;
      d[rl] = v[u].y;
      d[ppitch] = v[u].z;
      d[ppitch + rl] = v[u].w;
    }
  } else {
    const float* in = a.in + fld * plane + p0 + c + static_cast<size_t>(j0) * nx;
    float* d = buf + lcol;
    for_iters<NIT>([&](int it) { d[it * LS] = in[static_cast<size_t>(it) * JS * nx]; });
  }
  __syncthreads();
  if (busy) {
    const double shift = a.shift[fld];
    const double inorm = 0.25 * static_cast<double>(nx) * n;
    EigenScale<NK> sc;
#pragma unroll
    for (int q = 0; q < NK; ++q) sc.ry[q] = static_cast<float>((ly[q] - shift) * inorm);
    sc.xa = static_cast<float>(lxa * inorm);
    sc.xb = static_cast<float>(lxb * inorm);
    sc.za = p0 + 2 * pr == 0;
    float* g2 = buf + static_cast<size_t>(pr) * ppitch;
    if constexpr (two) {
      // the side job's stores drain under the transforms (which issue no
      // global loads here: a wait on a load also waits on earlier stores)
      zero_job(a.zero, static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x,
               static_cast<size_t>(gridDim.x) * gridDim.y);
      pair2_dst_core<n / 64>(g2, l, tw, wt, sc);
      __syncthreads();   // both waves' outputs are the next transform's input
      pair2_dst_core<n / 64>(g2, l, tw, wt);
    } else {
      wave_dst_core<P>(g2, tw, wt, sc);
      wave_dst_core<P>(g2, tw, wt);
    }
  }
  __syncthreads();
  if (cont) {
    const size_t sb = fld * plane + static_cast<size_t>(strip) * 4 * n;
    float4* dst = reinterpret_cast<float4*>(a.out + sb);
    float4* dy = fld == 0 && a.out_dy ? reinterpret_cast<float4*>(a.out_dy + static_cast<size_t>(strip) * 4 * n)
                                      : nullptr;
    const float mihy = static_cast<float>(-0.5 / g.hy);
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const int j = tid + u * kBlock;
      const float* q = buf + Pd::ridx(j);
      dst[j] = float4{q[0], q[rl], q[ppitch], q[ppitch + rl]};
      if (dy) {
        // -d_y by central differences, zero on row 0 and beyond row n - 1
        // (neighbour indices clamped into the strip)
        const float* qu = buf + Pd::ridx(j + 1 < n ? j + 1 : j);
        const float* qd = buf + Pd::ridx(j > 0 ? j - 1 : 0);
        const bool hu = j + 1 < n, in = j > 0;
        float4 d4;
        d4.x = in ? mihy * ((hu ? qu[0] : 0.f) - qd[0]) : 0.f;
        d4.y = in ? mihy * ((hu ? qu[rl] : 0.f) - qd[rl]) : 0.f;
        d4.z = in ? mihy * ((hu ? qu[ppitch] : 0.f) - qd[ppitch]) : 0.f;
        d4.w = in ? mihy * ((hu ? qu[ppitch + rl] : 0.f) - qd[ppitch + rl]) : 0.f;
        dy[j] = d4;
      }
    }
    return;
  }
  float* out = a.out + fld * plane + p0 + c + static_cast<size_t>(j0) * nx;
  const float* r = buf + lcol;
  if (fld == 0 && a.out_dy) {
    // -d_y by central differences, zero on the boundary rows j = 0 and the
    // clamped neighbour beyond j = ny - 1; j + 1 (j - 1) crosses a padding
    // gap (4 words) exactly when j0 + 1 (j0) is a multiple of 32
    float* dy = a.out_dy + p0 + c + static_cast<size_t>(j0) * nx;
    const float mihy = static_cast<float>(-0.5 / g.hy);
    const int up = Pd::ridx(j0 + 1) - Pd::ridx(j0), dn = Pd::ridx(j0 - 1) - Pd::ridx(j0);
    for_iters<NIT>([&](int it) {
      const float* q = r + it * LS;
      const int j = j0 + it * JS;
      // the neighbour reads stay inside the strip (clamped at the two ends)
      const float v = q[0];
      const float vu = j + 1 < n ? q[it == NIT - 1 && j0 == JS - 1 ? 0 : up] : 0.f;
      const float vd = j > 0 ? q[it == 0 && j0 == 0 ? 0 : dn] : 0.f;
      out[static_cast<size_t>(it) * JS * nx] = v;
      dy[static_cast<size_t>(it) * JS * nx] = j > 0 ? mihy * (vu - vd) : 0.f;
    });
  } else {
    for_iters<NIT>([&](int it) { out[static_cast<size_t>(it) * JS * nx] = r[it * LS]; });
  }
}

// DST along y, eigenvalue division, inverse DST along y (and -d_y for
// field 0 when requested) of column strip `strip` of field fld.
template <typename T, int LOGN>
__device__ __forceinline__ void col_block(const Geom& g, const ColArgs<T>& a,
                                          const AxisTables<T>& ty, const double* __restrict__ lamx,
                                          int strip, int fld, unsigned char* smem_raw) {
  if constexpr (fast_core(sizeof(T), 1 << LOGN) && core_lanes(sizeof(T), 1 << LOGN) == 128) {
    col_block_core<LOGN, 4>(g, a, ty, lamx, strip, fld, smem_raw);   // the launcher checks w = 4
    return;
  } else if constexpr (fast_core(sizeof(T), 1 << LOGN)) {
    if (a.w == 8)
      col_block_core<LOGN, 8>(g, a, ty, lamx, strip, fld, smem_raw);
    else if (a.w == 4)
      col_block_core<LOGN, 4>(g, a, ty, lamx, strip, fld, smem_raw);
    else
      col_block_core<LOGN, 2>(g, a, ty, lamx, strip, fld, smem_raw);
    return;
  }
  __syncthreads();   // the workgroup's previous use of LDS is complete
  T* buf = reinterpret_cast<T*>(smem_raw);
  const int ny = g.ny, nx = g.nx;
  const int W = a.w;
  const int ppitch = pair_pitch<T>(ny);
  const int p0 = strip * W;
  unsigned char* tbase = smem_raw + static_cast<size_t>(W / 2) * ppitch * sizeof(T);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables<T, LOGN>(ty, tbase, tw, pre);
  double* slamx = reinterpret_cast<double*>(tbase + table_bytes<T>(ny));   // the strip's
  const double* slam = ty.lam;                                              // x, y eigenvalues
  if constexpr (!fast_core(sizeof(T), 1 << LOGN)) {
    stage_doubles<(1 << LOGN)>(slamx, ty.lam);
    slam = slamx;
    slamx += ny;
  }
  if (static_cast<int>(threadIdx.x) < W) slamx[threadIdx.x] = lamx[strip * W + threadIdx.x];
  const size_t plane = static_cast<size_t>(nx) * ny;
  const T* in = a.in + fld * plane;
  const int lw = 31 - __clz(W), ly = g.ly;
  for_elems<32>(W * ny, [&](int e) {
    const int c = e & (W - 1), j = e >> lw;
    buf[Pad<T>::rpos(ny, ppitch, c, j)] = in[j * nx + p0 + c];
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.ly, W, ppitch, tw, pre);
  const double shift = a.shift[fld];
  // 1 / normalisation (nx ny / 4, exact): the eigenvalue sum in FP64 without
  // a division, the one division in the field precision
  const double inorm = 0.25 * static_cast<double>(nx) * ny;
  for_elems(W * ny, [&](int e) {
    const int c = e >> ly, q = e & (ny - 1);
    const int p = p0 + c;
    T* r = buf + Pad<T>::rpos(ny, ppitch, c, 0);
    const int iq = Pad<T>::ridx(q);
    const T den = static_cast<T>((slamx[c] + slam[q] - shift) * inorm);
    const T v = r[iq] / den;
    r[iq] = (p > 0 && q > 0) ? v : T(0);
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
template <typename T, int LOGN, int RC>
__device__ __forceinline__ void row_inv_pc_block(const Geom& g, const PCArgs<T>& a,
                                                 const AxisTables<T>& tx, int bxi, int fld,
                                                 unsigned char* smem_raw) {
  __syncthreads();   // the workgroup's previous use of LDS is complete
  T* buf = reinterpret_cast<T*>(smem_raw);
  constexpr int n = 1 << LOGN;   // = nx
  const int R = RC > 0 ? RC : g.rr;
  const int ppitch = pair_pitch<T>(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables<T, LOGN>(tx, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int j0 = bxi * R;
  plane_to_rows<T, RC, LOGN>(g, R, j0, a.in + static_cast<size_t>(fld) * g.nx * g.ny, buf, ppitch);
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  T* b = fld == 0 ? a.bx : a.by;
  T* tp = fld == 0 ? a.tape_bx : a.tape_by;
  double dsum = 0.0, nsum = 0.0;
  for_row_elems<RC, LOGN, 32>(R, [&](int e) {
    const int r = e >> LOGN, i = e & (n - 1);
    const int j = j0 + r;
    const T v = buf[RowLay<T, LOGN>::rpos(n, ppitch, r, i)];
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
// two in FP32 with the half-length transform and four in FP64 (measured at
// 1024^2), four with the FP32 core (two pairs of two waves at 1024).
template <typename T>
int row_rows(int nx, int ny) {
  if (core_lanes(sizeof(T), nx) == 128) return 4;   // two-wave core: two pairs per workgroup
  const bool core = fast_core(sizeof(T), nx);
  const int per = nx >= 512 || core ? 1 : 512 / nx;
  const int waves = nx <= 512 ? 1 : (sizeof(T) == 8 || core ? 4 : 2);
  int r = 2 * per * dst_detail::pass_waves("QSP_ROW_WAVES", waves);
  if (r > ny) r = ny;
  if (r > 2 * per * (kBlock / 64)) r = 2 * per * (kBlock / 64);   // one pair group per wave
  while (r > 2 && dst_detail::pass_lds<T>(r, nx) > 147456) r >>= 1;
  return r;
}

}  // namespace qsp
