// Batched 2D Dirichlet solve that allocates no device memory: the
// transforms' intermediate planes and their tables live in one file-scope
// static device array per GPU instead of a context's buffers (for callers
// that cannot allocate: code under stream capture, tight serving loops).
// Same three sine-transform passes as qsp_solve_poisson (fast Poisson
// solver of HiPACE++, arXiv:2109.10277 Sec. III.B), run in place.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "kernels.hpp"
#include "runtime.hpp"

namespace {

// Planes of the solve (nbatch x nx x ny values of the field precision), then
// the two axes' tables.
constexpr size_t kPlaneBytes = size_t(16) << 20;
constexpr size_t kTableBytes = size_t(256) << 10;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kPlaneBytes + kTableBytes];

std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};   // device address of `scratch`, per GPU

// Address of this device's copy of `scratch` (the device must be current).
unsigned char* scratch_on(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw qsp::DeviceError(std::string("hipGetSymbolAddress(scratch) failed: ") +
                             hipGetErrorString(e));
    g_ptr[device] = static_cast<unsigned char*>(p);
  }
  return g_ptr[device];
}

// The transform tables of one axis (layout as the context's, see
// AxisTables), computed on the device, one thread per entry.
template <typename T>
__global__ void k_axis_tables(int n, double h, qsp::Cplx<T>* tw, T* pre, double* lam) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= 2 * n) return;
  double s, c;
  if (qsp::fast_core(sizeof(T), n)) {
    const int NL = qsp::core_lanes(sizeof(T), n);
    const int k1 = m / NL, l = m % NL;
    sincospi(-2.0 * static_cast<double>((l * k1) % (2 * n)) / (2 * n), &s, &c);
    tw[m] = {static_cast<T>(c), static_cast<T>(s)};
    if (m < NL / 8 * 9) {
      auto* w = reinterpret_cast<qsp::Cplx<T>*>(pre);
      const int la = m / 9, c1 = m % 9;
      sincospi(-2.0 * (la * c1) / static_cast<double>(NL), &s, &c);
      w[m] = c1 < 8 ? qsp::Cplx<T>{static_cast<T>(c), static_cast<T>(s)}
                    : qsp::Cplx<T>{T(0), T(0)};
    }
  } else if (m < n) {
    sincospi(-2.0 * m / n, &s, &c);
    tw[m] = {static_cast<T>(c), static_cast<T>(s)};
    pre[m] = static_cast<T>(sinpi(static_cast<double>(m) / n));
  }
  if (m < n) {
    const double q = sinpi(0.5 * m / n);
    lam[m] = -4.0 / (h * h) * q * q;
  }
}

template <typename T>
size_t axis_table_bytes(int n) {
  return static_cast<size_t>(n) * (2 * sizeof(qsp::Cplx<T>) + sizeof(T) + sizeof(double));
}

template <typename T>
qsp::AxisTables<T> axis_at(unsigned char* base, int n) {
  auto* tw = reinterpret_cast<qsp::Cplx<T>*>(base);
  auto* pre = reinterpret_cast<T*>(base + static_cast<size_t>(n) * 2 * sizeof(qsp::Cplx<T>));
  auto* lam = reinterpret_cast<double*>(base + static_cast<size_t>(n) *
                                                   (2 * sizeof(qsp::Cplx<T>) + sizeof(T)));
  return {tw, pre, lam};
}

template <typename T>
void solve(const qsp_config& c, unsigned char* ptr, int nb, const T* src, T* dst, double shift,
           hipStream_t st) {
  using namespace qsp;
  Geom g{};
  g.nx = c.nx;
  g.ny = c.ny;
  for (g.lx = 0; (1 << g.lx) < c.nx; ++g.lx) {}
  for (g.ly = 0; (1 << g.ly) < c.ny; ++g.ly) {}
  g.x_lo = c.x_lo;
  g.y_lo = c.y_lo;
  g.hx = (c.x_hi - c.x_lo) / c.nx;
  g.hy = (c.y_hi - c.y_lo) / c.ny;
  g.rr = row_rows<T>(c.nx, c.ny);
  g.order = 1;
  g.strip = 0;   // the passes run in place: the planes stay row-major
  const size_t pl = static_cast<size_t>(c.nx) * c.ny;
  const size_t nn = static_cast<size_t>(c.nx + 1) * (c.ny + 1);
  T* planes = reinterpret_cast<T*>(ptr);
  unsigned char* tab = ptr + kPlaneBytes;
  // tables are 8-byte aligned pieces: x axis first, then y
  const AxisTables<T> tx = axis_at<T>(tab, c.nx);
  const AxisTables<T> ty = axis_at<T>(tab + axis_table_bytes<T>(c.nx), c.ny);
  hipLaunchKernelGGL(k_axis_tables<T>, dim3((2 * c.nx + 255) / 256), dim3(256), 0, st, c.nx, g.hx,
                     const_cast<Cplx<T>*>(tx.tw), const_cast<T*>(tx.pre),
                     const_cast<double*>(tx.lam));
  QSP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_axis_tables<T>, dim3((2 * c.ny + 255) / 256), dim3(256), 0, st, c.ny, g.hy,
                     const_cast<Cplx<T>*>(ty.tw), const_cast<T*>(ty.pre),
                     const_cast<double*>(ty.lam));
  QSP_LAUNCH_CHECK();
  for (int b = 0; b < nb; ++b) launch_from_nodes<T, T>(g, src + b * nn, planes + b * pl, st);
  // each pass reads its rows or column strips into LDS before writing them
  // back, so all three run in place
  RowInvArgs<T> r{};
  for (int b = 0; b < nb; ++b) {
    r.in[b] = planes + b * pl;
    r.out[b] = planes + b * pl;
  }
  launch_row_inv<T>(g, r, nb, tx, st);
  ColArgs<T> col{};
  col.in = planes;
  col.out = planes;
  for (int b = 0; b < 4; ++b) col.shift[b] = shift;
  col.w = col_width<T>(g, nb);
  launch_col_solve<T>(g, col, nb, ty, tx.lam, nullptr, st);
  launch_row_inv<T>(g, r, nb, tx, st);
  for (int b = 0; b < nb; ++b) launch_to_nodes_t<T>(g, planes + b * pl, dst + b * nn, st);
}

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

}  // namespace

namespace qsp {

qsp_status solve_poisson_noalloc(const qsp_config* cfg, int device, void* stream, int nbatch,
                                 const void* src, void* dst, double shift, std::string& err) {
  if (!cfg) return err = "null config", QSP_ERR_INVALID_ARG;
  const qsp_config& c = *cfg;
  if (!pow2_in(c.nx, 16, 2048) || !pow2_in(c.ny, 16, 2048))
    return err = "nx and ny must be powers of two in [16, 2048]", QSP_ERR_INVALID_ARG;
  if (!(std::isfinite(c.x_lo) && std::isfinite(c.x_hi) && c.x_hi > c.x_lo &&
        std::isfinite(c.y_lo) && std::isfinite(c.y_hi) && c.y_hi > c.y_lo))
    return err = "box extents must be finite with hi > lo", QSP_ERR_INVALID_ARG;
  if (c.precision != QSP_FP32 && c.precision != QSP_FP64)
    return err = "precision must be QSP_FP32 or QSP_FP64", QSP_ERR_INVALID_ARG;
  if (nbatch < 1 || nbatch > 4) return err = "nbatch must be 1..4", QSP_ERR_INVALID_ARG;
  if (!(shift >= 0.0) || !std::isfinite(shift))
    return err = "shift must be finite and >= 0", QSP_ERR_INVALID_ARG;
  if (!src || !dst) return err = "null src or dst", QSP_ERR_INVALID_ARG;
  const size_t es = c.precision == QSP_FP64 ? sizeof(double) : sizeof(float);
  const size_t need = static_cast<size_t>(nbatch) * c.nx * c.ny * es;
  if (need > kPlaneBytes)
    return err = "nbatch * nx * ny values (" + std::to_string(need) +
                 " bytes) exceed the static scratch of " + std::to_string(kPlaneBytes) +
                 " bytes",
           QSP_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev ||
      device >= kMaxDevices)
    return err = "no such HIP device", QSP_ERR_INVALID_ARG;
  try {
    QSP_HIP(hipSetDevice(device));
    unsigned char* ptr = scratch_on(device);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (c.precision == QSP_FP64)
      solve<double>(c, ptr, nbatch, static_cast<const double*>(src), static_cast<double*>(dst),
                    shift, st);
    else
      solve<float>(c, ptr, nbatch, static_cast<const float*>(src), static_cast<float*>(dst),
                   shift, st);
  } catch (const std::exception& e) {
    err = e.what();
    return QSP_ERR_DEVICE;
  }
  return QSP_OK;
}

}  // namespace qsp
