// Batched 2D Dirichlet Poisson / Helmholtz solve kernels and their launchers
// (fast Poisson solver of HiPACE++, arXiv:2109.10277 Sec. III.B).  The
// transform machinery and the per-block bodies live in dst_impl.hpp.
#include "dst_impl.hpp"

namespace qsp {

using namespace dst_detail;

// ---------------------------------------------------------------------------
// P1: sources + forward DST along x
// ---------------------------------------------------------------------------

// field ids of the psi / Ez / Bz batch
template <typename T, int LOGN, int RC>
__global__ void __launch_bounds__(kBlock, dst_blocks_per_cu(LOGN, sizeof(T)))
k_src_fwd_pez(Geom g, SrcPEZ<T> a, AxisTables<T> tx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  constexpr int n = 1 << LOGN;   // = nx
  const int R = RC > 0 ? RC : g.rr;
  const int ppitch = pair_pitch<T>(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables<T, LOGN>(tx, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  // neighbouring row blocks share the 128-byte lines of strip-ordered
  // planes: keep them on one XCD (one L2)
  const int j0 = xcd_strip(blockIdx.x, gridDim.x) * R;
  const int fld = blockIdx.y;   // 0 psi, 1 Ez, 2 Bz
  const double ihx = 0.5 / g.hx, ihy = 0.5 / g.hy;
  // neighbour indices are clamped so that every load is in bounds; values
  // outside the interior are replaced by selects
  for_row_elems<RC, LOGN>(R, [&](int e) {
    const int r = e >> LOGN, i = e & (n - 1);
    const int j = j0 + r;
    const int o = j * n + i;
    double s;
    if (fld == 0) {
      s = -(a.rho_mjz[o] + (a.ionx ? a.n0 * a.ionx[i] * a.iony[j] : a.n0));
    } else {
      const int ow = i > 0 ? o - 1 : o, oe = i + 1 < n ? o + 1 : o;
      const int os = j > 0 ? o - n : o, on = j + 1 < g.ny ? o + n : o;
      const double xe = a.jx[oe], xw = a.jx[ow], xn = a.jx[on], xs = a.jx[os];
      const double ye = a.jy[oe], yw = a.jy[ow], yn = a.jy[on], ys = a.jy[os];
      const double jx_e = i + 1 < n ? xe : 0.0, jy_e = i + 1 < n ? ye : 0.0;
      const double jx_n = j + 1 < g.ny ? xn : 0.0, jy_n = j + 1 < g.ny ? yn : 0.0;
      s = fld == 1 ? (jx_e - xw) * ihx + (jy_n - ys) * ihy : (jx_n - xs) * ihy - (jy_e - yw) * ihx;
    }
    buf[RowLay<T, LOGN>::rpos(n, ppitch, r, i)] = static_cast<T>((i > 0 && j > 0) ? s : 0.0);
  });
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  rows_to_plane<T, RC, LOGN>(g, R, j0, buf, ppitch, a.out + static_cast<size_t>(fld) * g.nx * g.ny);
}

template <typename T, int LOGN, int RC>
__global__ void __launch_bounds__(kBlock, dst_blocks_per_cu(LOGN, sizeof(T)))
k_src_fwd_bxby(Geom g, SrcBxBy<T> a, AxisTables<T> tx, const DevCounters* ctr) {
  if (ctr->pc_done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  src_bxby_block<T, LOGN, RC>(g, a, tx, xcd_strip(blockIdx.x, gridDim.x), blockIdx.y, smem_raw);
}

// ---------------------------------------------------------------------------
// P2: column strip solve
// ---------------------------------------------------------------------------
template <typename T, int LOGN>
__global__ void __launch_bounds__(kBlock, col_blocks_per_cu(LOGN, sizeof(T)))
k_col_solve(Geom g, ColArgs<T> a, AxisTables<T> ty, const double* __restrict__ lamx,
            const DevCounters* ctr) {
  if (a.honor_done && ctr->pc_done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  col_block<T, LOGN>(g, a, ty, lamx, xcd_strip(blockIdx.x, gridDim.x), blockIdx.y, smem_raw);
  // the side job's stores come last (the memory counter the strip load waits
  // on also counts stores); the two-wave core's pass issues them itself,
  // before its transforms
  if constexpr (core_lanes(sizeof(T), 1 << LOGN) != 128)
    zero_job(a.zero, static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x,
             static_cast<size_t>(gridDim.x) * gridDim.y);
}

// ---------------------------------------------------------------------------
// P3: inverse DST along x with epilogues
// ---------------------------------------------------------------------------
template <typename T, int LOGN, int RC>
__global__ void __launch_bounds__(kBlock, dst_blocks_per_cu(LOGN, sizeof(T)))
k_row_inv(Geom g, RowInvArgs<T> a, AxisTables<T> tx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  constexpr int n = 1 << LOGN;   // = nx
  const int R = RC > 0 ? RC : g.rr;
  const int ppitch = pair_pitch<T>(n);
  const Cplx<T>* tw;
  const T* pre;
  stage_tables<T, LOGN>(tx, smem_raw + static_cast<size_t>(R / 2) * ppitch * sizeof(T), tw, pre);
  const int j0 = xcd_strip(blockIdx.x, gridDim.x) * R;   // neighbours on one XCD
  const int fld = blockIdx.y;
  {
    Geom gi = g;
    gi.strip = a.in_strip;
    plane_to_rows<T, RC, LOGN>(gi, R, j0, a.in[fld], buf, ppitch);
  }
  __syncthreads();
  block_dst<T, LOGN>(buf, g.lx, R, ppitch, tw, pre);
  guess_job(a.guess, static_cast<size_t>(g.nx) * g.ny);
  T* out = a.out[fld];
  T* out_dx = a.out_dx[fld];
  if (a.out_strip) {   // an intermediate plane (no -d_x)
    Geom go = g;
    go.strip = 1;
    rows_to_plane<T, RC, LOGN>(go, R, j0, buf, ppitch, out);
    return;
  }
  const T mihx = static_cast<T>(-0.5 / g.hx);
  for_row_elems<RC, LOGN>(R, [&](int e) {
    const int r = e >> LOGN, i = e & (n - 1);
    const int j = j0 + r;
    const T* row = buf + RowLay<T, LOGN>::rpos(n, ppitch, r, 0);
    const T u = row[RowLay<T, LOGN>::ridx(i)];
    out[j * n + i] = j > 0 ? u : T(0);
    if (out_dx) {
      const T ue = row[RowLay<T, LOGN>::ridx(i + 1 < n ? i + 1 : i)], uw = row[RowLay<T, LOGN>::ridx(i > 0 ? i - 1 : 0)];
      const T d = mihx * ((i + 1 < n ? ue : T(0)) - uw);
      out_dx[j * n + i] = (i > 0 && j > 0) ? d : T(0);
    }
  });
}

template <typename T, int LOGN, int RC>
__global__ void __launch_bounds__(kBlock, dst_blocks_per_cu(LOGN, sizeof(T)))
k_row_inv_pc(Geom g, PCArgs<T> a, AxisTables<T> tx, DevCounters* ctr) {
  if (ctr->pc_done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  row_inv_pc_block<T, LOGN, RC>(g, a, tx, xcd_strip(blockIdx.x, gridDim.x), blockIdx.y, smem_raw);
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

// Each wave transforms one group of row pairs (one pair for the FP32 core,
// max(1, 512/n) otherwise; two waves per pair at 1024 with the FP32 core,
// exactly two pairs): a pass must not give a workgroup more rows.
// The strip order of the intermediate planes moves 4 rows x 4 columns at a
// time: it needs 4-row row blocks and 4-column column strips.
static void check_strip(const Geom& g, int rows_or_cols) {
  if (g.strip && rows_or_cols != 4)
    throw std::invalid_argument("transform pass: strip-ordered planes need blocks of 4 rows or columns");
}

template <typename T>
static void check_rows(int n, int rows) {
  if (core_lanes(sizeof(T), n) == 128) {   // the two-wave core needs all four waves busy
    if (rows != 4) throw std::invalid_argument("transform pass: the two-wave core takes 4 rows");
    return;
  }
  const int per = fast_core(sizeof(T), n) || n >= 512 ? 1 : 512 / n;
  if (rows > 2 * per * (kBlock / 64))
    throw std::invalid_argument("transform pass: more row pairs than its waves take");
}

template <typename T>
void launch_src_fwd_pez(const Geom& g, const SrcPEZ<T>& a, const AxisTables<T>& tx,
                        hipStream_t st) {
  const int R = g.rr;
  check_rows<T>(g.nx, R);
  check_strip(g, R);
  const size_t lds = static_cast<size_t>(R / 2) * pair_pitch<T>(g.nx) * sizeof(T) + table_bytes<T>(g.nx);
  with_logn(g.nx, [&](auto e) {
    constexpr int E = decltype(e)::value;
    with_rows<T, E>(R, [&](auto rc) {
      constexpr int RC = decltype(rc)::value;
      allow_lds(reinterpret_cast<const void*>(&k_src_fwd_pez<T, E, RC>), lds);
      hipLaunchKernelGGL((k_src_fwd_pez<T, E, RC>), dim3(g.ny / R, 3), dim3(kBlock), lds, st, g, a, tx);
    });
  });
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_src_fwd_bxby(const Geom& g, const SrcBxBy<T>& a, const AxisTables<T>& tx,
                         const DevCounters* ctr, hipStream_t st) {
  const int R = g.rr;
  check_rows<T>(g.nx, R);
  check_strip(g, R);
  const size_t lds = static_cast<size_t>(R / 2) * pair_pitch<T>(g.nx) * sizeof(T) + table_bytes<T>(g.nx);
  with_logn(g.nx, [&](auto e) {
    constexpr int E = decltype(e)::value;
    with_rows<T, E>(R, [&](auto rc) {
      constexpr int RC = decltype(rc)::value;
      allow_lds(reinterpret_cast<const void*>(&k_src_fwd_bxby<T, E, RC>), lds);
      hipLaunchKernelGGL((k_src_fwd_bxby<T, E, RC>), dim3(g.ny / R, 2), dim3(kBlock), lds, st, g, a, tx,
                         ctr);
    });
  });
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_col_solve(const Geom& g, const ColArgs<T>& a, int nfield, const AxisTables<T>& ty,
                      const double* lamx, const DevCounters* ctr, hipStream_t st) {
  const int W = a.w;
  if (W < 2 || (W & (W - 1)) || g.nx % W || nfield < 1 || nfield > 4)
    throw std::invalid_argument("column pass: bad strip width or field count");
  check_rows<T>(g.ny, W);
  check_strip(g, W);
  const size_t lds = static_cast<size_t>(W / 2) * pair_pitch<T>(g.ny) * sizeof(T) + table_bytes<T>(g.ny) +
                     lam_bytes<T>(g.ny, W);
  with_logn(g.ny, [&](auto e) {
    constexpr int E = decltype(e)::value;
    allow_lds(reinterpret_cast<const void*>(&k_col_solve<T, E>), lds);
    hipLaunchKernelGGL((k_col_solve<T, E>), dim3(g.nx / W, nfield), dim3(kBlock), lds, st, g, a,
                       ty, lamx, ctr);
  });
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_row_inv(const Geom& g, const RowInvArgs<T>& a, int nfield, const AxisTables<T>& tx,
                    hipStream_t st) {
  const int R = g.rr;
  check_rows<T>(g.nx, R);
  check_strip(g, R);
  const size_t lds = static_cast<size_t>(R / 2) * pair_pitch<T>(g.nx) * sizeof(T) + table_bytes<T>(g.nx);
  with_logn(g.nx, [&](auto e) {
    constexpr int E = decltype(e)::value;
    with_rows<T, E>(R, [&](auto rc) {
      constexpr int RC = decltype(rc)::value;
      allow_lds(reinterpret_cast<const void*>(&k_row_inv<T, E, RC>), lds);
      hipLaunchKernelGGL((k_row_inv<T, E, RC>), dim3(g.ny / R, nfield), dim3(kBlock), lds, st, g, a, tx);
    });
  });
  QSP_LAUNCH_CHECK();
}

template <typename T>
void launch_row_inv_pc(const Geom& g, const PCArgs<T>& a, const AxisTables<T>& tx,
                       DevCounters* ctr, hipStream_t st) {
  const int R = g.rr;
  check_rows<T>(g.nx, R);
  check_strip(g, R);
  const size_t lds = static_cast<size_t>(R / 2) * pair_pitch<T>(g.nx) * sizeof(T) + table_bytes<T>(g.nx);
  with_logn(g.nx, [&](auto e) {
    constexpr int E = decltype(e)::value;
    with_rows<T, E>(R, [&](auto rc) {
      constexpr int RC = decltype(rc)::value;
      allow_lds(reinterpret_cast<const void*>(&k_row_inv_pc<T, E, RC>), lds);
      hipLaunchKernelGGL((k_row_inv_pc<T, E, RC>), dim3(g.ny / R, 2), dim3(kBlock), lds, st, g, a, tx,
                         ctr);
    });
  });
  QSP_LAUNCH_CHECK();
}

int pc_partial_count(const Geom& g) { return 2 * (g.ny / g.rr); }

template <typename T>
int col_width(const Geom& g, int nfield) {
  return col_strip<T>(g.nx, g.ny, nfield);
}
template int col_width<float>(const Geom&, int);
template int col_width<double>(const Geom&, int);
template int row_rows<float>(int, int);
template int row_rows<double>(int, int);

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
