// Host runtime of libqsp: buffers, tables and the per-slice schedule of the
// quasi-static PIC loop (HiPACE++, arXiv:2109.10277, Sec. II slice routine
// with the Sec. III.B predictor-corrector for Bx/By).
#include "runtime.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>

namespace qsp {

namespace {

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
bool finite(double v) { return std::isfinite(v); }

}  // namespace

double default_pc_shift(double n0) { return 0.5 * kAB5[0] * n0; }

namespace {
template <int O>
void deposit_lattice_point(int c, double t, int n, double scale, std::vector<double>& f) {
  int b = 0;
  const double d = shape::locate<O>(c, t, n, b);
  double w[O + 1];
  shape::weights<O>(d, w);
  for (int a = 0; a <= O; ++a)
    if (b + a >= 1 && b + a < n) f[b + a] += w[a] * scale;
}
}  // namespace

std::vector<double> ion_profile(int n, int ppc, int order) {
  // The ions sit on the electrons' rest lattice, c + (q + 1/2)/ppc in node
  // units, and are deposited with the same shape; along one axis node i
  // receives 1/ppc times the sum of the shape weights.  Boundary nodes are
  // Dirichlet nodes and carry no source.
  std::vector<double> f(n + 1, 0.0);
  with_order(order, [&](auto o) {
    constexpr int O = decltype(o)::value;
    for (int c = 0; c < n; ++c)
      for (int q = 0; q < ppc; ++q)
        deposit_lattice_point<O>(c, (2.0 * q + 1.0) / (2.0 * ppc), n, 1.0 / ppc, f);
  });
  return f;
}

std::string validate(const qsp_config& c) {
  if (!pow2(c.nx) || c.nx < 16 || c.nx > 2048) return "nx must be a power of two in [16, 2048]";
  if (!pow2(c.ny) || c.ny < 16 || c.ny > 2048) return "ny must be a power of two in [16, 2048]";
  if (!finite(c.x_lo) || !finite(c.x_hi) || !(c.x_hi > c.x_lo)) return "need finite x_lo < x_hi";
  if (!finite(c.y_lo) || !finite(c.y_hi) || !(c.y_hi > c.y_lo)) return "need finite y_lo < y_hi";
  if (c.nzeta < 1) return "nzeta must be >= 1";
  if (c.precision != QSP_FP32 && c.precision != QSP_FP64) return "precision must be QSP_FP32 or QSP_FP64";
  if (!finite(c.zeta_hi)) return "zeta_hi must be finite";
  if (!finite(c.dzeta) || !(c.dzeta > 0)) return "dzeta must be finite and > 0";
  if (!(c.ppc_x == 1 || c.ppc_x == 2 || c.ppc_x == 4)) return "ppc_x must be 1, 2 or 4";
  if (!(c.ppc_y == 1 || c.ppc_y == 2 || c.ppc_y == 4)) return "ppc_y must be 1, 2 or 4";
  if (!finite(c.n0) || !(c.n0 > 0)) return "n0 must be finite and > 0";
  if (c.pc_max_iter < 1 || c.pc_max_iter > 1000) return "pc_max_iter must be in [1, 1000]";
  if (!finite(c.pc_tol)) return "pc_tol must be finite";
  if (!finite(c.pc_shift)) return "pc_shift must be finite (< 0 selects the default)";
  if (!finite(c.psi_floor) || !(c.psi_floor > 0) || !(c.psi_floor < 1)) return "psi_floor must be in (0, 1)";
  if (c.mem_cap_bytes < 0) return "mem_cap_bytes must be >= 0";
  if (c.deposit_mode != 0 && c.deposit_mode != 1) return "deposit_mode must be 0 or 1";
  if (c.shape_order < 0 || c.shape_order > 3) return "shape_order must be 0, 1, 2 or 3";
  if (c.bxby_solver != QSP_BXBY_PC && c.bxby_solver != QSP_BXBY_EXPLICIT)
    return "bxby_solver must be QSP_BXBY_PC or QSP_BXBY_EXPLICIT";
  if (c.bxby_solver == QSP_BXBY_EXPLICIT && c.shape_order < 1)
    return "the explicit Bx/By solver needs shape_order 1, 2 or 3";
  return "";
}

int64_t device_bytes_needed(const qsp_config& c) {
  const int64_t ts = c.precision == QSP_FP64 ? 8 : 4;
  const int64_t plane = static_cast<int64_t>(c.nx) * c.ny;
  const int64_t np = static_cast<int64_t>(c.nx) * c.ppc_x * c.ny * c.ppc_y;
  int64_t b = 0;
  b += plane * ts * (5 + 6 + 8);                 // fields, B history, DST scratch
  b += plane * 8 * (3 * 5 + 2);                  // deposits, trial currents
  b += np * ts * (6 + 20);                       // particle SoA + history
  if (c.bxby_solver != QSP_BXBY_EXPLICIT) b += np * ts * 6;   // trial record
  b += (c.nx + c.ny) * (3 * ts + 8 + 8) + 4096;  // tables, counters
  b += (c.nx + c.ny + 2) * 8;                    // ion profile
  if (c.bxby_solver == QSP_BXBY_EXPLICIT) b += plane * 8 * 13 + 4096;   // explicit solver
  b += static_cast<int64_t>(c.ny) * 16 + 64;     // residual partials
  return b;
}

// HIP-event timers around kernel launches, per kernel class.
class KernelTimer {
 public:
  ~KernelTimer() {
    for (auto& e : pool_) (void)hipEventDestroy(e);
    for (auto& p : pending_) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
  }
  void reset(int every) {
    every_ = every;
    std::fill(std::begin(ms_), std::end(ms_), 0.0);
    std::fill(std::begin(n_), std::end(n_), 0);
  }
  bool active(int k) const { return every_ > 0 && k % every_ == 0; }
  int every() const { return every_; }
  void begin(int cls, hipStream_t st) {
    cur_ = {get(), get(), cls};
    QSP_HIP(hipEventRecord(cur_.a, st));
  }
  void end(hipStream_t st) {
    QSP_HIP(hipEventRecord(cur_.b, st));
    pending_.push_back(cur_);
  }
  // synchronises on the recorded events and folds them into the totals
  void collect() {
    for (auto& p : pending_) {
      QSP_HIP(hipEventSynchronize(p.b));
      float ms = 0.f;
      QSP_HIP(hipEventElapsedTime(&ms, p.a, p.b));
      ms_[p.cls] += ms;
      n_[p.cls] += 1;
      pool_.push_back(p.a);
      pool_.push_back(p.b);
    }
    pending_.clear();
  }
  void read(qsp_kernel_times* out) {
    collect();
    for (int c = 0; c < QSP_NK; ++c) {
      out->ms[c] = ms_[c];
      out->launches[c] = n_[c];
    }
  }

 private:
  struct Pair {
    hipEvent_t a, b;
    int cls;
  };
  hipEvent_t get() {
    if (pool_.empty()) {
      hipEvent_t e;
      QSP_HIP(hipEventCreate(&e));
      return e;
    }
    hipEvent_t e = pool_.back();
    pool_.pop_back();
    return e;
  }
  int every_ = 0;
  double ms_[QSP_NK] = {};
  int64_t n_[QSP_NK] = {};
  Pair cur_{};
  std::vector<Pair> pending_;
  std::vector<hipEvent_t> pool_;
};

// Per-slice record of the forward pass kept for the reverse pass: the state
// at the start of the slice, its fields and every predictor-corrector
// iterate B^0 .. B^M.
template <typename T>
struct TapeSlot {
  Particles<T> p;
  T* f[5];        // psi, Ex-By, Ey+Bx, Ez, Bz
  T* b;           // [pc_max_iter + 1][2][plane]
  T* rec;         // the slice's trial record [6][np]
};

// Full slice state at the start of a chunk of slices.
template <typename T>
struct Checkpoint {
  Particles<T> p;
  double* j[2];   // J_perp of the previous slice
  T* b[4];        // Bx, By of the previous slice, then of the one before
};

template <typename T>
class Box final : public BoxBase {
 public:
  Box(const qsp_config& cfg, int device, hipStream_t st) : st_(st), device_(device) {
    cfg_ = cfg;
    geom_.nx = cfg.nx;
    geom_.ny = cfg.ny;
    geom_.lx = ilog2i(cfg.nx);
    geom_.ly = ilog2i(cfg.ny);
    geom_.x_lo = cfg.x_lo;
    geom_.y_lo = cfg.y_lo;
    geom_.hx = (cfg.x_hi - cfg.x_lo) / cfg.nx;
    geom_.hy = (cfg.y_hi - cfg.y_lo) / cfg.ny;
    geom_.rr = row_rows<T>(cfg.nx, cfg.ny);
    geom_.order = cfg.shape_order;
    // both axes on the two-wave core at 1024 points: strip-ordered
    // intermediate planes
    geom_.strip = core_lanes(sizeof(T), cfg.nx) == 128 && core_lanes(sizeof(T), cfg.ny) == 128 &&
                  cfg.nx >= 1024 && cfg.ny >= 1024;
    lat_.ppc_x = cfg.ppc_x;
    lat_.ppc_y = cfg.ppc_y;
    lat_.nX = cfg.nx * cfg.ppc_x;
    lat_.nY = cfg.ny * cfg.ppc_y;
    lat_.np = static_cast<int64_t>(lat_.nX) * lat_.nY;
    explicit_ = cfg.bxby_solver == QSP_BXBY_EXPLICIT;
    // predictor-corrector screening, or the explicit solver's preconditioner
    // shift (the unperturbed plasma's chi = n0)
    shift_ = cfg.pc_shift >= 0 ? cfg.pc_shift : (explicit_ ? cfg.n0 : default_pc_shift(cfg.n0));
    tiled_ = cfg.deposit_mode == 0;
    tile_rows_ = default_tile_rows();
    real_tile_rows_ = default_tile_rows(4096);
    tile_halo_ = default_tile_halo();
    if (const char* e = std::getenv("QSP_GRAPH")) graphs_ = std::atoi(e) != 0;   // 0: launch eagerly
    // QSP_PC_BUDGET: 0 switches the speculative P-C budgets off; -1 launches
    // one iteration fewer than the learned budgets (where that leaves at
    // least one), also with a moving beam, so that boxes are run twice: a
    // test of the rerun path
    if (const char* e = std::getenv("QSP_PC_BUDGET")) spec_mode_ = std::atoi(e);
    QSP_HIP(hipSetDevice(device_));
    try {
      allocate();
      build_tables();
      QSP_HIP(hipEventCreate(&ev0_));
      QSP_HIP(hipEventCreate(&ev1_));
    } catch (...) {
      release();
      throw;
    }
  }

  ~Box() override {
    free_graph(graph_);
    free_graph(graph_b_);
    if (cap_st_) (void)hipStreamDestroy(cap_st_);
    free_beam();
    free_adjoint();
    clear_beam_currents();
    release();
  }

  void set_deposit_tiled(bool on) override {
    if (on != tiled_ && trial_[0]) {
      // with tiles the trial pushes store every node of the trial current
      // planes and add into the shared ones, without tiles they add into
      // the trial current planes: either way from zero
      QSP_HIP(hipSetDevice(device_));
      launch_zero(trial_[0], plane(), st_);
      launch_zero(trial_[1], plane(), st_);
      zero_shared();
    }
    tiled_ = on;
    ++launch_version_;
  }
  void set_timing(int every) override {
    timer_.collect();
    if (every != timer_.every()) ++launch_version_;   // the sampled launches change
    timer_.reset(every);
  }
  void get_kernel_times(qsp_kernel_times* out) override { timer_.read(out); }

  // ---------------------------------------------------------------- state
  void init_plasma() override {
    QSP_HIP(hipSetDevice(device_));
    rec_valid_ = false;
    resort_beam();
    reset_box();
    box_reruns_ = 0;
    fresh_box_ = true;
  }

  // plasma at rest ahead of the box, every field, deposit and counter zero
  void reset_box() {
    launch_init_plasma<T>(lat_, p_, cfg_.n0 / (cfg_.ppc_x * cfg_.ppc_y), st_);
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 2; ++c) launch_zero_t<T>(b_[b][c], plane(), st_);
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 5; ++c) launch_zero(dep_[d][c], plane(), st_);
    launch_zero(trial_[0], plane(), st_);
    launch_zero(trial_[1], plane(), st_);
    zero_shared();
    launch_zero_t<T>(t1_, 4 * plane(), st_);
    launch_zero_t<T>(t2_, 4 * plane(), st_);
    static_assert(sizeof(DevCounters) % sizeof(double) == 0, "counter block size");
    launch_zero_t<double>(reinterpret_cast<double*>(ctr_), sizeof(DevCounters) / sizeof(double),
                          st_);
    cursor_ = 0;
    dep_valid_ = false;
    initialised_ = true;
    slices_done_ = 0;
    dst_solves_ = 0;
    pushes_ = 0;
    // every buffer is clear: start the rotations from one fixed state, so
    // that each box from the head launches the same sequence
    ip_ = 0, ic_ = 1, in_ = 2;
    ik_ = 0, i1_ = 1, i2_ = 2;
  }

  // A beam pushed during a box is sorted by slice again before the next box
  // (its particles keep their slice for the whole of a box).
  void resort_beam() {
    if (beam_n_ == 0 || !beam_dirty_) return;
    QSP_HIP(hipMemcpyAsync(beam_tmp_, beam_soa_, 7 * beam_n_ * sizeof(float),
                           hipMemcpyDeviceToDevice, st_));
    beam_sort(beam_tmp_, beam_soa_, beam_n_, cfg_.zeta_hi, cfg_.dzeta, cfg_.nzeta, bs_, beam_off_,
              st_);
    beam_dirty_ = false;
  }

  void set_beam_gaussian(const double* amp, double sx, double sy, double x0,
                         double y0) override {
    rec_valid_ = false;
    ++launch_version_;
    amp_.assign(amp, amp + cfg_.nzeta);
    // profile factors and their derivatives with respect to sigma
    std::vector<double> gx(cfg_.nx + 1, 0.0), gy(cfg_.ny + 1, 0.0);
    std::vector<double> dgx(cfg_.nx + 1, 0.0), dgy(cfg_.ny + 1, 0.0);
    for (int i = 1; i < cfg_.nx; ++i) {
      const double x = cfg_.x_lo + i * geom_.hx - x0;
      gx[i] = std::exp(-x * x / (2.0 * sx * sx));
      dgx[i] = gx[i] * x * x / (sx * sx * sx);
    }
    for (int j = 1; j < cfg_.ny; ++j) {
      const double y = cfg_.y_lo + j * geom_.hy - y0;
      gy[j] = std::exp(-y * y / (2.0 * sy * sy));
      dgy[j] = gy[j] * y * y / (sy * sy * sy);
    }
    QSP_HIP(hipMemcpyAsync(bgx_, gx.data(), gx.size() * sizeof(double), hipMemcpyHostToDevice, st_));
    QSP_HIP(hipMemcpyAsync(bgy_, gy.data(), gy.size() * sizeof(double), hipMemcpyHostToDevice, st_));
    QSP_HIP(hipMemcpyAsync(dbgx_, dgx.data(), dgx.size() * sizeof(double), hipMemcpyHostToDevice, st_));
    QSP_HIP(hipMemcpyAsync(dbgy_, dgy.data(), dgy.size() * sizeof(double), hipMemcpyHostToDevice, st_));
    QSP_HIP(hipStreamSynchronize(st_));
    has_gauss_ = true;
  }

  void set_beam_particles(int64_t n, const float* soa, double dt) override {
    QSP_HIP(hipSetDevice(device_));
    rec_valid_ = false;
    ++launch_version_;
    free_beam();
    if (n == 0) return;
    const int nz = cfg_.nzeta;
    if (nz + 1 > kMaxBeamKeys) throw std::invalid_argument("particle beams need nzeta < 16384");
    const int nchunk = beam_sort_chunks(n);
    const int64_t need = n * (14 * 4) + static_cast<int64_t>(nchunk + 1) * (nz + 1) * 4 +
                         static_cast<int64_t>(nz + 2) * 8;
    if (cfg_.mem_cap_bytes > 0 && bytes_ + need > cfg_.mem_cap_bytes) throw std::bad_alloc();
    beam_soa_ = beam_alloc<float>(7 * n);
    beam_tmp_ = beam_alloc<float>(7 * n);
    bs_.hist = beam_alloc<int>(static_cast<size_t>(nchunk) * (nz + 1));
    bs_.total = beam_alloc<int>(nz + 1);
    bs_.off = beam_alloc<int64_t>(nz + 2);
    bs_.nchunk = nchunk;
    beam_n_ = n;
    beam_dt_ = dt;
    moving_beam_ = dt != 0.0;
    beam_sort(soa, beam_soa_, n, cfg_.zeta_hi, cfg_.dzeta, nz, bs_, beam_off_, st_);
    beam_dirty_ = false;
  }

  void get_beam_particles(float* soa) override {
    QSP_HIP(hipMemcpyAsync(soa, beam_soa_, 7 * beam_n_ * sizeof(float), hipMemcpyDeviceToDevice, st_));
    QSP_HIP(hipStreamSynchronize(st_));
  }

  int64_t beam_count() const override { return beam_n_; }

  void set_beam_current(int k, const double* jz) override {
    QSP_HIP(hipSetDevice(device_));
    rec_valid_ = false;
    ++launch_version_;
    if (cur_.empty()) cur_.assign(cfg_.nzeta, nullptr);
    if (!jz) {
      if (cur_[k]) {
        QSP_HIP(hipStreamSynchronize(st_));
        QSP_HIP(hipFree(cur_[k]));
        cur_[k] = nullptr;
        const int64_t b = static_cast<int64_t>(std::max<size_t>(plane() * sizeof(double), 256));
        bytes_ -= b;
      }
      return;
    }
    if (!cur_[k]) {
      const size_t bytes = std::max<size_t>(plane() * sizeof(double), 256);
      if (cfg_.mem_cap_bytes > 0 && bytes_ + static_cast<int64_t>(bytes) > cfg_.mem_cap_bytes)
        throw std::bad_alloc();
      void* p = nullptr;
      const hipError_t e = hipMalloc(&p, bytes);
      if (e == hipErrorOutOfMemory) throw std::bad_alloc();
      QSP_HIP(e);
      cur_[k] = static_cast<double*>(p);
      bytes_ += static_cast<int64_t>(bytes);
    }
    launch_from_nodes<double, double>(geom_, jz, cur_[k], st_);
  }

  void clear_beam_currents() override {
    ++launch_version_;
    if (cur_.empty()) return;
    (void)hipStreamSynchronize(st_);
    const int64_t b = static_cast<int64_t>(std::max<size_t>(plane() * sizeof(double), 256));
    for (double*& p : cur_)
      if (p) {
        (void)hipFree(p);
        p = nullptr;
        bytes_ -= b;
      }
    rec_valid_ = false;
  }

  void get_stats(qsp_stats* s) override {
    DevCounters c{};
    QSP_HIP(hipMemcpyAsync(&c, ctr_, sizeof(c), hipMemcpyDeviceToHost, st_));
    QSP_HIP(hipStreamSynchronize(st_));
    std::memset(s, 0, sizeof(*s));
    s->slices = slices_done_;
    s->particle_pushes = pushes_;
    s->pc_iterations = static_cast<int64_t>(c.pc_iterations);
    s->pc_not_converged = static_cast<int64_t>(c.pc_not_converged);
    s->n_clamped = static_cast<int64_t>(c.n_clamped);
    s->n_absorbed = static_cast<int64_t>(c.n_absorbed);
    s->n_deposit_global = static_cast<int64_t>(c.n_dep_global);
    s->dst_solves = dst_solves_ + 2 * static_cast<int64_t>(c.pc_iterations);
    s->max_pc_residual = c.max_resid;
    s->elapsed_ms = last_ms_;
    s->device_bytes = bytes_;
    s->box_reruns = box_reruns_;
    nonfinite_ = c.nonfinite != 0;
  }

  bool check_nonfinite() override {
    DevCounters c{};
    QSP_HIP(hipMemcpyAsync(&c, ctr_, sizeof(c), hipMemcpyDeviceToHost, st_));
    QSP_HIP(hipStreamSynchronize(st_));
    return c.nonfinite != 0;
  }

  void get_state(qsp_slice_state* d) override {
    const size_t np = static_cast<size_t>(lat_.np);
    const size_t nn = nodes();
    double* tmp = nullptr;
    const size_t tot = np * 26 + 6 * nn;
    QSP_HIP(hipMalloc(&tmp, tot * sizeof(double)));
    try {
      double* q = tmp;
      double *x = q, *y = q + np, *ux = q + 2 * np, *uy = q + 3 * np, *ps = q + 4 * np,
             *w = q + 5 * np, *h = q + 6 * np;
      double* g = q + 26 * np;
      launch_export_state<T>(geom_, lat_, p_, x, y, ux, uy, ps, w, h, cursor_, st_);
      to_nodes_d(dep_[ip_][1], g);
      to_nodes_d(dep_[ip_][2], g + nn);
      launch_to_nodes<T>(geom_, b_[i1_][0], g + 2 * nn, st_);
      launch_to_nodes<T>(geom_, b_[i1_][1], g + 3 * nn, st_);
      launch_to_nodes<T>(geom_, b_[i2_][0], g + 4 * nn, st_);
      launch_to_nodes<T>(geom_, b_[i2_][1], g + 5 * nn, st_);
      auto d2h = [&](double* dst, const double* src, size_t n) {
        QSP_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToHost, st_));
      };
      d2h(d->x, x, np);
      d2h(d->y, y, np);
      d2h(d->ux, ux, np);
      d2h(d->uy, uy, np);
      d2h(d->psi, ps, np);
      d2h(d->w, w, np);
      d2h(d->hist, h, 20 * np);
      d2h(d->jx_prev, g, nn);
      d2h(d->jy_prev, g + nn, nn);
      d2h(d->bx_prev1, g + 2 * nn, nn);
      d2h(d->by_prev1, g + 3 * nn, nn);
      d2h(d->bx_prev2, g + 4 * nn, nn);
      d2h(d->by_prev2, g + 5 * nn, nn);
      QSP_HIP(hipStreamSynchronize(st_));
      d->k = cursor_;
    } catch (...) {
      (void)hipFree(tmp);
      throw;
    }
    QSP_HIP(hipFree(tmp));
  }

  void set_state(const qsp_slice_state* s) override {
    fresh_box_ = false;
    resort_beam();
    const size_t np = static_cast<size_t>(lat_.np);
    const size_t nn = nodes();
    double* tmp = nullptr;
    const size_t tot = np * 26 + 6 * nn;
    QSP_HIP(hipMalloc(&tmp, tot * sizeof(double)));
    try {
      double* q = tmp;
      auto h2d = [&](double* dst, const double* src, size_t n) {
        QSP_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, st_));
      };
      h2d(q, s->x, np);
      h2d(q + np, s->y, np);
      h2d(q + 2 * np, s->ux, np);
      h2d(q + 3 * np, s->uy, np);
      h2d(q + 4 * np, s->psi, np);
      h2d(q + 5 * np, s->w, np);
      h2d(q + 6 * np, s->hist, 20 * np);
      double* g = q + 26 * np;
      h2d(g, s->jx_prev, nn);
      h2d(g + nn, s->jy_prev, nn);
      h2d(g + 2 * nn, s->bx_prev1, nn);
      h2d(g + 3 * nn, s->by_prev1, nn);
      h2d(g + 4 * nn, s->bx_prev2, nn);
      h2d(g + 5 * nn, s->by_prev2, nn);
      launch_import_state<T>(geom_, lat_, p_, q, q + np, q + 2 * np, q + 3 * np, q + 4 * np,
                             q + 5 * np, q + 6 * np, s->k, cfg_.dzeta, st_);
      for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 5; ++c) launch_zero(dep_[d][c], plane(), st_);
      launch_zero(trial_[0], plane(), st_);
      launch_zero(trial_[1], plane(), st_);
      zero_shared();
      launch_from_nodes<double, double>(geom_, g, dep_[ip_][1], st_);
      launch_from_nodes<double, double>(geom_, g + nn, dep_[ip_][2], st_);
      launch_from_nodes<double, T>(geom_, g + 2 * nn, b_[i1_][0], st_);
      launch_from_nodes<double, T>(geom_, g + 3 * nn, b_[i1_][1], st_);
      launch_from_nodes<double, T>(geom_, g + 4 * nn, b_[i2_][0], st_);
      launch_from_nodes<double, T>(geom_, g + 5 * nn, b_[i2_][1], st_);
      QSP_HIP(hipStreamSynchronize(st_));
    } catch (...) {
      (void)hipFree(tmp);
      throw;
    }
    QSP_HIP(hipFree(tmp));
    cursor_ = s->k;
    dep_valid_ = false;
    initialised_ = true;
    rec_valid_ = false;
  }

  void solve_poisson(int nb, const void* src, void* dst, double shift) override {
    QSP_HIP(hipSetDevice(device_));
    const size_t pl = plane(), nn = nodes();
    const T* s = static_cast<const T*>(src);
    T* d = static_cast<T*>(dst);
    for (int b = 0; b < nb; ++b) launch_from_nodes<T, T>(geom_, s + b * nn, t2_ + b * pl, st_);
    RowInvArgs<T> r{};
    for (int b = 0; b < nb; ++b) {
      r.in[b] = t2_ + b * pl;
      r.out[b] = t1_ + b * pl;
    }
    r.out_strip = geom_.strip;
    launch_row_inv<T>(geom_, r, nb, tx(), st_);
    ColArgs<T> c{};
    c.in = t1_;
    c.out = t2_;
    for (int b = 0; b < 4; ++b) c.shift[b] = shift;
    c.w = col_width<T>(geom_, nb);
    launch_col_solve<T>(geom_, c, nb, ty(), lamx_, ctr_, st_);
    for (int b = 0; b < nb; ++b) {
      r.in[b] = t2_ + b * pl;
      r.out[b] = t1_ + b * pl;
    }
    r.in_strip = geom_.strip;
    r.out_strip = 0;
    launch_row_inv<T>(geom_, r, nb, tx(), st_);
    for (int b = 0; b < nb; ++b) launch_to_nodes_t<T>(geom_, t1_ + b * pl, d + b * nn, st_);
  }

  // ---------------------------------------------------------------- loop
  void advance_slice(const qsp_slice_out* out) override {
    QSP_HIP(hipSetDevice(device_));
    rec_valid_ = false;
    fresh_box_ = false;
    OutCopy oc{};
    if (out) {
      for (int q = 0; q < QSP_NQ; ++q)
        if (out->q[q]) add_out(oc, q, out->q[q], 0);
    }
    step(oc, nullptr, nullptr);
  }

  void run_box(const qsp_box_out* out) override {
    QSP_HIP(hipSetDevice(device_));
    rec_valid_ = false;
    const bool fresh = fresh_box_;
    fresh_box_ = false;
    if (graph_eligible()) {
      run_box_graphs(out, fresh);
      return;
    }
    QSP_HIP(hipEventRecord(ev0_, st_));
    box_loop(out);
    QSP_HIP(hipEventRecord(ev1_, st_));
    QSP_HIP(hipEventSynchronize(ev1_));
    float ms = 0.f;
    QSP_HIP(hipEventElapsedTime(&ms, ev0_, ev1_));
    last_ms_ = ms;
  }

 private:
  void box_loop(const qsp_box_out* out) {
    const int k0 = cursor_;
    while (cursor_ < cfg_.nzeta) {
      const int rel = cursor_ - k0;
      OutCopy oc = box_outputs(out, rel);
      step(oc, out && out->pc_iters ? out->pc_iters + rel : nullptr,
           out && out->pc_resid ? out->pc_resid + rel : nullptr);
    }
  }

  // Whole boxes from HIP graphs.  With the predictor-corrector to a
  // tolerance, a box started from a fresh plasma launches per slice only as
  // many iterations as the budget of the slice holds instead of
  // pc_max_iter (the launches after convergence would read the device's
  // converged flag and return).  A budget is the most iterations the slice
  // needed in the boxes run so far, plus one where the slice's count has
  // risen before.  A slice that ends its budget unconverged below
  // pc_max_iter is counted on the device; the box is then run again from
  // its start (plasma reset, a macro-particle beam restored) with every
  // iteration launched, so that results and iteration counts are always
  // those of the full launch sequence.  Boxes whose beam moves between them
  // differ from box to box (the per-slice counts of the paper-scale step
  // change by one here and there every time step), so they launch every
  // iteration: a rerun costs a whole box and would outweigh what the
  // budgets save there.
  void run_box_graphs(const qsp_box_out* out, bool fresh) {
    const bool moving = beam_n_ > 0 && beam_dt_ != 0.0;
    const bool pc = !explicit_ && cfg_.pc_tol > 0.0 && spec_mode_ != 0 && (!moving || spec_mode_ < 0);
    const bool spec = pc && fresh && budget_ready_ && budget_version_ == launch_version_;
    bool fell_short = false;
    if (spec) {
      const HostState h0 = save_host();
      if (moving)
        QSP_HIP(hipMemcpyAsync(beam_tmp_, beam_soa_, 7 * beam_n_ * sizeof(float),
                               hipMemcpyDeviceToDevice, st_));
      set_budget_launch();
      budget_on_ = true;
      try {
        if (!graph_matches(graph_b_, out)) build_graph(graph_b_, out);
        replay_graph(graph_b_);
      } catch (...) {
        budget_on_ = false;
        throw;
      }
      budget_on_ = false;
      unsigned int shortfall = 0;
      QSP_HIP(hipMemcpy(&shortfall, &ctr_->budget_short, sizeof(shortfall), hipMemcpyDeviceToHost));
      if (shortfall == 0) return;
      fell_short = true;
      ++box_reruns_;
      restore_host(h0);
      if (moving)
        QSP_HIP(hipMemcpyAsync(beam_soa_, beam_tmp_, 7 * beam_n_ * sizeof(float),
                               hipMemcpyDeviceToDevice, st_));
      reset_box();
    }
    if (!graph_matches(graph_, out)) build_graph(graph_, out);
    replay_graph(graph_);
    if (pc && fresh) {
      learn_budgets(fell_short);
      // capture the speculative box now, from this box's start, so that the
      // next box only replays it
      const HostState end = save_host();
      restore_host(graph_.start);
      set_budget_launch();
      budget_on_ = true;
      try {
        if (!graph_matches(graph_b_, out)) build_graph(graph_b_, out);
      } catch (...) {
        budget_on_ = false;
        restore_host(end);
        throw;
      }
      budget_on_ = false;
      restore_host(end);
    }
  }

  // the iterations a speculative box launches per slice
  void set_budget_launch() {
    budget_launch_.resize(cfg_.nzeta);
    for (int k = 0; k < cfg_.nzeta; ++k) {
      int b = budget_[k] + margin_[k];
      if (spec_mode_ < 0) b = budget_[k] - 1;   // test of the rerun path
      budget_launch_[k] = std::max(1, std::min(b, cfg_.pc_max_iter));
    }
  }

  // budgets from the iteration counts of the box just run (a whole box from
  // a fresh plasma with every iteration launched); after a shortfall the
  // slices that needed more than they were given get a margin from now on
  void learn_budgets(bool after_shortfall) {
    std::vector<int32_t> it(cfg_.nzeta);
    QSP_HIP(hipMemcpy(it.data(), iters_own_, it.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (!budget_ready_ || budget_version_ != launch_version_) {
      budget_.assign(cfg_.nzeta, 1);
      margin_.assign(cfg_.nzeta, 0);
    }
    budget_version_ = launch_version_;
    for (int k = 0; k < cfg_.nzeta; ++k) {
      const int v = std::max(1, std::min(static_cast<int>(it[k]), cfg_.pc_max_iter));
      if (after_shortfall && spec_mode_ > 0 && v > budget_launch_[k]) margin_[k] = 1;
      budget_[k] = std::max(budget_[k], v);
    }
    budget_ready_ = true;
  }

  // ------------------------------------------------------- graph replay
  // A box run from the head launches the same ~24 kernels per slice every
  // time; it is captured once into HIP graphs and replayed, which halves the
  // per-launch overhead.  The launches that the kernel timer samples (the
  // real push) run outside the graphs between graph segments, so that
  // their events bracket exactly one kernel.  Everything that changes what a
  // box launches bumps launch_version_ and forces a new capture.
  struct HostState {
    int cursor, ip, ic, in, ik, i1, i2;
    bool dep_valid, beam_dirty, beam_ahead;
    int64_t slices, pushes, dst;
  };
  struct GraphItem {
    hipGraphExec_t exec;
    std::function<void()> eager;
    int cls;
  };
  struct BoxGraph {
    bool valid = false;
    uint64_t version = 0;
    bool has_out = false;
    qsp_box_out out{};
    HostState start{}, end{};
    std::vector<GraphItem> items;
    bool budgeted = false;          // captured with the speculative P-C budgets
    std::vector<int> budget;
  };

  HostState save_host() const {
    return {cursor_, ip_, ic_, in_, ik_, i1_, i2_, dep_valid_, beam_dirty_, beam_ahead_,
            slices_done_, pushes_, dst_solves_};
  }
  void restore_host(const HostState& h) {
    cursor_ = h.cursor;
    ip_ = h.ip, ic_ = h.ic, in_ = h.in;
    ik_ = h.ik, i1_ = h.i1, i2_ = h.i2;
    dep_valid_ = h.dep_valid;
    beam_dirty_ = h.beam_dirty;
    beam_ahead_ = h.beam_ahead;
    slices_done_ = h.slices;
    pushes_ = h.pushes;
    dst_solves_ = h.dst;
  }
  static bool same_host(const HostState& a, const HostState& b) {
    return a.cursor == b.cursor && a.ip == b.ip && a.ic == b.ic && a.in == b.in &&
           a.ik == b.ik && a.i1 == b.i1 && a.i2 == b.i2 && a.dep_valid == b.dep_valid &&
           a.beam_ahead == b.beam_ahead;
  }

  // whole boxes from the head (macro-particle beams included: their kernels
  // read the slice ranges of the current sort on the device)
  bool graph_eligible() const { return graphs_ && cursor_ == 0 && tape_slot_ == nullptr; }

  bool graph_matches(const BoxGraph& G, const qsp_box_out* out) const {
    if (!G.valid || G.version != launch_version_) return false;
    if (G.has_out != (out != nullptr)) return false;
    if (out && std::memcmp(&G.out, out, sizeof(qsp_box_out)) != 0) return false;
    if (G.budgeted != budget_on_ || (budget_on_ && G.budget != budget_launch_)) return false;
    const HostState h = save_host();
    return same_host(G.start, h) && G.start.slices == h.slices && G.start.pushes == h.pushes &&
           G.start.dst == h.dst;
  }

  void begin_segment() {
    QSP_HIP(hipStreamBeginCapture(st_, hipStreamCaptureModeRelaxed));
  }
  void end_segment() {
    hipGraph_t g = nullptr;
    QSP_HIP(hipStreamEndCapture(st_, &g));
    size_t nodes = 0;
    QSP_HIP(hipGraphGetNodes(g, nullptr, &nodes));
    if (nodes > 0) {
      hipGraphExec_t ge = nullptr;
      const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      QSP_HIP(e);
      cap_graph_->items.push_back({ge, {}, 0});
    } else {
      (void)hipGraphDestroy(g);
    }
  }

  // The capture runs on a stream of the library's own (the caller's stream
  // may be the legacy default stream, which cannot be captured); the graphs
  // are then launched on the caller's stream.
  void build_graph(BoxGraph& G, const qsp_box_out* out) {
    free_graph(G);
    cap_graph_ = &G;
    if (!cap_st_) QSP_HIP(hipStreamCreateWithFlags(&cap_st_, hipStreamNonBlocking));
    QSP_HIP(hipStreamSynchronize(st_));
    const HostState s0 = save_host();
    hipStream_t user = st_;
    st_ = cap_st_;
    capturing_ = true;
    try {
      begin_segment();
      box_loop(out);
      end_segment();
    } catch (...) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(st_, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(st_, &g);
        if (g) (void)hipGraphDestroy(g);
      }
      st_ = user;
      capturing_ = false;
      restore_host(s0);
      free_graph(G);
      throw;
    }
    st_ = user;
    capturing_ = false;
    G.end = save_host();
    restore_host(s0);
    G.start = s0;
    G.version = launch_version_;
    G.has_out = out != nullptr;
    G.out = out ? *out : qsp_box_out{};
    G.budgeted = budget_on_;
    G.budget = budget_on_ ? budget_launch_ : std::vector<int>{};
    G.valid = true;
  }

  void replay_graph(BoxGraph& G) {
    QSP_HIP(hipEventRecord(ev0_, st_));
    for (auto& it : G.items) {
      if (it.exec) {
        QSP_HIP(hipGraphLaunch(it.exec, st_));
      } else {
        timer_.begin(it.cls, st_);
        it.eager();
        timer_.end(st_);
      }
    }
    QSP_HIP(hipEventRecord(ev1_, st_));
    QSP_HIP(hipEventSynchronize(ev1_));
    float ms = 0.f;
    QSP_HIP(hipEventElapsedTime(&ms, ev0_, ev1_));
    last_ms_ = ms;
    restore_host(G.end);
  }

  void free_graph(BoxGraph& G) {
    for (auto& it : G.items)
      if (it.exec) (void)hipGraphExecDestroy(it.exec);
    G.items.clear();
    G.valid = false;
  }

 public:
  // ---------------------------------------------------------------- adjoint
  // Device bytes of the checkpoints, the tape of one chunk and the reverse
  // work space for a record of n_slices slices with checkpoints every K.
  int64_t adjoint_bytes(int n_slices, int K) const override {
    const int64_t ts = sizeof(T), pl = static_cast<int64_t>(plane()), np = lat_.np;
    const int64_t nck = (n_slices - 1) / K;
    const int64_t slots = std::min(K, n_slices);
    const int64_t part = 26 * np * ts;
    const int64_t ck = part + 2 * pl * 8 + 4 * pl * ts;
    const int64_t slot = part + 6 * np * ts + 5 * pl * ts + 2 * (cfg_.pc_max_iter + 1) * pl * ts;
    const int64_t work = 32 * np * ts + 18 * pl * 8 + 4 * static_cast<int64_t>(cfg_.nzeta) + 1024;
    return nck * ck + slots * slot + work + 256 * (8 * (nck + slots) + 32);
  }

  void record(int n_slices, int K, const qsp_box_out* out) override {
    fresh_box_ = false;
    QSP_HIP(hipSetDevice(device_));
    rec_valid_ = false;
    ensure_adjoint(n_slices, K);
    const int last0 = ((n_slices - 1) / K) * K;   // first slice of the last chunk
    QSP_HIP(hipEventRecord(ev0_, st_));
    while (cursor_ < n_slices) {
      const int k = cursor_;
      if (k % K == 0 && k < last0) save_checkpoint(k / K);
      OutCopy oc = box_outputs(out, k);
      TapeSlot<T>* slot = k >= last0 ? &tape_[k - last0] : nullptr;
      taped_step(oc, slot, out && out->pc_resid ? out->pc_resid + k : nullptr);
    }
    if (out && out->pc_iters)
      QSP_HIP(hipMemcpyAsync(out->pc_iters, iters_dev_, n_slices * sizeof(int32_t),
                             hipMemcpyDeviceToDevice, st_));
    read_iterations(last0, n_slices);
    QSP_HIP(hipEventRecord(ev1_, st_));
    QSP_HIP(hipEventSynchronize(ev1_));
    float ms = 0.f;
    QSP_HIP(hipEventElapsedTime(&ms, ev0_, ev1_));
    last_ms_ = ms;
    rec_slices_ = n_slices;
    rec_K_ = K;
    rec_valid_ = true;
  }

  void adjoint(const qsp_box_cotangent* cot, double* grad_amp, double* grad_sigma,
               double* loss) override {
    QSP_HIP(hipSetDevice(device_));
    const int n_slices = rec_slices_, K = rec_K_;
    const int nchunks = (n_slices - 1) / K + 1;
    const size_t pl = plane(), np = static_cast<size_t>(lat_.np);
    QSP_HIP(hipEventRecord(ev0_, st_));
    launch_zero(grad_amp, cfg_.nzeta, st_);
    launch_zero(grad_sigma, 2, st_);
    if (loss) launch_zero(loss, 1, st_);
    launch_zero_t<T>(lam_y_, 5 * np, st_);
    launch_zero_t<T>(lam_ring_, 20 * np, st_);
    for (double* q : {carry_j_[0], carry_j_[1], carry_b1_[0], carry_b1_[1], carry_b2_[0], carry_b2_[1]})
      launch_zero(q, pl, st_);
    for (int c = nchunks - 1; c >= 0; --c) {
      const int k0 = c * K, k1 = std::min(k0 + K, n_slices);
      if (c != nchunks - 1) {
        // recompute the chunk from its checkpoint, taping every slice
        restore_checkpoint(c);
        while (cursor_ < k1) {
          OutCopy oc{};
          taped_step(oc, &tape_[cursor_ - k0], nullptr);
        }
        read_iterations(k0, k1);
      }
      for (int k = k1 - 1; k >= k0; --k)
        reverse_slice(k, tape_[k - k0], cot, k == n_slices - 1, grad_amp, grad_sigma, loss);
    }
    QSP_HIP(hipEventRecord(ev1_, st_));
    QSP_HIP(hipEventSynchronize(ev1_));
    float ms = 0.f;
    QSP_HIP(hipEventElapsedTime(&ms, ev0_, ev1_));
    last_ms_ = ms;
    // the tape and the plasma now hold an intermediate state
    rec_valid_ = false;
    initialised_ = false;
  }

 private:
  size_t plane() const { return static_cast<size_t>(cfg_.nx) * cfg_.ny; }

  // output copies of slice rel (relative to the first slice of the run)
  OutCopy box_outputs(const qsp_box_out* out, int rel) {
    OutCopy oc{};
    if (!out) return oc;
    const int every = out->stack_every > 0 ? out->stack_every : 1;
    const size_t nn = nodes();
    for (int q = 0; q < QSP_NQ; ++q) {
      const size_t es = elem_size(q);
      if (out->stack[q] && rel % every == 0)
        add_out(oc, q, static_cast<char*>(out->stack[q]) + (rel / every) * nn * es, 0);
      if (out->lineout[q])
        add_out(oc, q, static_cast<char*>(out->lineout[q]) + rel * (cfg_.nx + 1) * es, 1);
      if (out->axis[q]) add_out(oc, q, static_cast<char*>(out->axis[q]) + rel * es, 2);
    }
    return oc;
  }

  // ------------------------------------------------------- adjoint storage
  template <typename U>
  U* adj_alloc(size_t n) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(n * sizeof(U), 256);
    const hipError_t e = hipMalloc(&p, bytes);
    if (e == hipErrorOutOfMemory) throw std::bad_alloc();
    QSP_HIP(e);
    adj_allocs_.push_back(p);
    bytes_ += static_cast<int64_t>(bytes);
    adj_bytes_ += static_cast<int64_t>(bytes);
    return static_cast<U*>(p);
  }

  void free_adjoint() {
    (void)hipStreamSynchronize(st_);
    for (void* p : adj_allocs_) (void)hipFree(p);
    adj_allocs_.clear();
    bytes_ -= adj_bytes_;
    adj_bytes_ = 0;
    ckpt_.clear();
    tape_.clear();
    adj_shape_ = {0, 0};
    rec_valid_ = false;
  }

  Particles<T> alloc_particles() {
    const size_t np = static_cast<size_t>(lat_.np);
    Particles<T> q{};
    T* base = adj_alloc<T>(26 * np);
    q.xi_x = base;
    q.xi_y = base + np;
    q.ux = base + 2 * np;
    q.uy = base + 3 * np;
    q.psi = base + 4 * np;
    q.w = base + 5 * np;
    q.hist = base + 6 * np;
    return q;
  }

  // (re)allocates checkpoints, tape and reverse work space for (n_slices, K)
  void ensure_adjoint(int n_slices, int K) {
    const int nck = (n_slices - 1) / K;
    const int slots = std::min(K, n_slices);
    if (adj_shape_.first == nck && adj_shape_.second == slots) return;
    free_adjoint();
    if (cfg_.mem_cap_bytes > 0 && bytes_ + adjoint_bytes(n_slices, K) > cfg_.mem_cap_bytes)
      throw std::bad_alloc();
    try {
      const size_t pl = plane(), np = static_cast<size_t>(lat_.np);
      for (int c = 0; c < nck; ++c) {
        Checkpoint<T> ck{};
        ck.p = alloc_particles();
        double* j = adj_alloc<double>(2 * pl);
        ck.j[0] = j;
        ck.j[1] = j + pl;
        T* b = adj_alloc<T>(4 * pl);
        for (int q = 0; q < 4; ++q) ck.b[q] = b + q * pl;
        ckpt_.push_back(ck);
      }
      for (int s = 0; s < slots; ++s) {
        TapeSlot<T> ts{};
        ts.p = alloc_particles();
        T* f = adj_alloc<T>(5 * pl);
        for (int q = 0; q < 5; ++q) ts.f[q] = f + q * pl;
        ts.b = adj_alloc<T>(2 * static_cast<size_t>(cfg_.pc_max_iter + 1) * pl);
        ts.rec = adj_alloc<T>(6 * np);
        tape_.push_back(ts);
      }
      lam_y_ = adj_alloc<T>(5 * np);
      lam_ring_ = adj_alloc<T>(20 * np);
      lam_acc_ = adj_alloc<T>(7 * np);
      double* w = adj_alloc<double>(18 * pl);
      for (int q = 0; q < 6; ++q) lam_f_[q] = w + q * pl;
      lam_psi_ = w + 6 * pl;
      lam_jz_ = w + 7 * pl;
      jp_[0] = w + 8 * pl;
      jp_[1] = w + 9 * pl;
      carry_j_[0] = w + 10 * pl;
      carry_j_[1] = w + 11 * pl;
      carry_b1_[0] = w + 12 * pl;
      carry_b1_[1] = w + 13 * pl;
      carry_b2_[0] = w + 14 * pl;
      carry_b2_[1] = w + 15 * pl;
      lam_b_[0] = w + 16 * pl;
      lam_b_[1] = w + 17 * pl;
      iters_dev_ = adj_alloc<int32_t>(cfg_.nzeta);
      iters_host_.assign(cfg_.nzeta, 0);
    } catch (...) {
      free_adjoint();
      throw;
    }
    if (cfg_.mem_cap_bytes > 0 && bytes_ > cfg_.mem_cap_bytes) {
      free_adjoint();
      throw std::bad_alloc();
    }
    adj_shape_ = {nck, slots};
  }

  void save_checkpoint(int c) {
    Checkpoint<T>& ck = ckpt_[c];
    launch_copy_particles<T>(lat_, p_, ck.p, cursor_, cfg_.dzeta, st_);
    CopyPlanes<double, double> j{};
    j.src[0] = dep_[ip_][1];
    j.src[1] = dep_[ip_][2];
    j.dst[0] = ck.j[0];
    j.dst[1] = ck.j[1];
    launch_copy_planes<double, double>(plane(), 2, j, st_);
    CopyPlanes<T, T> b{};
    b.src[0] = b_[i1_][0];
    b.src[1] = b_[i1_][1];
    b.src[2] = b_[i2_][0];
    b.src[3] = b_[i2_][1];
    for (int q = 0; q < 4; ++q) b.dst[q] = ck.b[q];
    launch_copy_planes<T, T>(plane(), 4, b, st_);
  }

  void restore_checkpoint(int c) {
    const Checkpoint<T>& ck = ckpt_[c];
    launch_copy_particles<T>(lat_, ck.p, p_, c * rec_K_, cfg_.dzeta, st_);
    CopyPlanes<double, double> j{};
    j.src[0] = ck.j[0];
    j.src[1] = ck.j[1];
    j.dst[0] = dep_[ip_][1];
    j.dst[1] = dep_[ip_][2];
    launch_copy_planes<double, double>(plane(), 2, j, st_);
    CopyPlanes<T, T> b{};
    for (int q = 0; q < 4; ++q) b.src[q] = ck.b[q];
    b.dst[0] = b_[i1_][0];
    b.dst[1] = b_[i1_][1];
    b.dst[2] = b_[i2_][0];
    b.dst[3] = b_[i2_][1];
    launch_copy_planes<T, T>(plane(), 4, b, st_);
    cursor_ = c * rec_K_;
    dep_valid_ = false;
  }

  // one forward slice; with a tape slot, also records what the reverse pass
  // of this slice reads
  void taped_step(OutCopy& oc, TapeSlot<T>* slot, double* resid_out) {
    const int k = cursor_;
    // the slice's first trial push copies the particle state into the slot,
    // so a tape needs the predictor-corrector
    if (slot && explicit_) throw std::logic_error("a taped slice needs the predictor-corrector");
    tape_slot_ = slot;
    step(oc, iters_dev_ + k, resid_out);
    tape_slot_ = nullptr;
    if (slot) {
      CopyPlanes<T, T> f{};
      const T* src[5] = {psi_, exmby_, eypbx_, ez_, bz_};
      for (int q = 0; q < 5; ++q) {
        f.src[q] = src[q];
        f.dst[q] = slot->f[q];
      }
      launch_copy_planes<T, T>(plane(), 5, f, st_);
    }
  }

  void read_iterations(int k0, int k1) {
    QSP_HIP(hipMemcpyAsync(iters_host_.data() + k0, iters_dev_ + k0, (k1 - k0) * sizeof(int32_t),
                           hipMemcpyDeviceToHost, st_));
    QSP_HIP(hipStreamSynchronize(st_));
  }

  T* tape_b(const TapeSlot<T>& t, int m, int c) const {
    return t.b + (2 * static_cast<size_t>(m) + c) * plane();
  }

  // (lap - shift)^-1 of nb planes staged in t2_; the solutions land in t1_
  void adj_solve(int nb, double shift) {
    const size_t pl = plane();
    RowInvArgs<T> r{};
    for (int b = 0; b < nb; ++b) {
      r.in[b] = t2_ + b * pl;
      r.out[b] = t1_ + b * pl;
    }
    r.out_strip = geom_.strip;
    launch_row_inv<T>(geom_, r, nb, tx(), st_);
    ColArgs<T> c{};
    c.in = t1_;
    c.out = t2_;
    for (int b = 0; b < 4; ++b) c.shift[b] = shift;
    c.honor_done = 0;
    c.w = col_width<T>(geom_, nb);
    launch_col_solve<T>(geom_, c, nb, ty(), lamx_, ctr_, st_);
    r.in_strip = geom_.strip;
    r.out_strip = 0;
    launch_row_inv<T>(geom_, r, nb, tx(), st_);
  }

  // Reverse pass of slice k: the transpose of step() taken in the opposite
  // order (real push, predictor-corrector iterations M-1 .. 0, initial
  // guess, psi/Ez/Bz solves, deposit), handing the adjoints of the state,
  // J_perp and B of slice k on to slice k-1.
  void reverse_slice(int k, const TapeSlot<T>& t, const qsp_box_cotangent* cot, bool last,
                     double* grad_amp, double* grad_sigma, double* loss) {
    const size_t pl = plane(), nn = nodes();
    const int M = iters_host_[k];
    if (M < 1 || M > cfg_.pc_max_iter)
      throw std::runtime_error("recorded predictor-corrector iteration count out of range");
    const bool has_cot = cot && k >= cot->k_lo;
    const T* bxM = tape_b(t, M, 0);
    const T* byM = tape_b(t, M, 1);
    // seed: cotangents of slice k, plus what slice k+1 handed to B_k
    {
      AdjSeedArgs<T> a{};
      for (int c = 0; c < 7; ++c)
        a.cot[c] = has_cot && cot->w[c]
                       ? static_cast<const T*>(cot->w[c]) + static_cast<size_t>(k - cot->k_lo) * nn
                       : nullptr;
      a.extra[QSP_BX] = carry_b1_[0];
      a.extra[QSP_BY] = carry_b1_[1];
      a.out[QSP_PSI] = lam_psi_;
      for (int c = 1; c < 7; ++c) a.out[c] = lam_f_[c - 1];
      a.zero[0] = lam_jz_;
      a.zero[1] = jp_[0];
      a.zero[2] = jp_[1];
      launch_adj_seed<T>(geom_, a, st_);
      if (has_cot && loss) {
        LossArgs<T> l{};
        const T* fld[7] = {t.f[0], t.f[1], t.f[2], t.f[3], bxM, byM, t.f[4]};
        for (int c = 0; c < 7; ++c) {
          l.cot[c] = a.cot[c];
          l.field[c] = fld[c];
        }
        l.loss = loss;
        launch_loss<T>(geom_, l, st_);
      }
    }
    AdjPushArgs<T> pa{};
    pa.p = t.p;
    pa.lam_y = lam_y_;
    pa.lam_ring = lam_ring_;
    pa.k = k;
    pa.dzeta = cfg_.dzeta;
    pa.hx = geom_.hx;
    pa.hy = geom_.hy;
    pa.psi_floor = cfg_.psi_floor;
    pa.inv2dz = 0.5 / cfg_.dzeta;
    pa.tile_rows = tile_rows_;
    pa.tile_halo = tile_halo_;
    // real push k -> k+1 (none after the last recorded slice)
    if (!last) {
      pa.f = {t.f[1], t.f[2], t.f[3], bxM, byM, t.f[4]};
      for (int c = 0; c < 6; ++c) pa.lam_F[c] = lam_f_[c];
      launch_adj_push<T>(geom_, lat_, pa, false, st_);
    }
    // predictor-corrector iterations in reverse; those after the first
    // transpose only what their own Bx, By change (the rest is summed per
    // particle and taken up by the first iteration's transpose)
    const double* lbx = lam_f_[3];
    const double* lby = lam_f_[4];
    pa.rec = t.rec;
    for (int m = M - 1; m >= 0; --m) {
      AdjSrcArgs<T> s{};
      s.count = 2;
      s.p0[0] = lbx;
      s.p0[1] = lby;
      s.c0[0] = s.c0[1] = 1.0;
      s.out[0] = t2_;
      s.out[1] = t2_ + pl;
      launch_adj_source<T>(geom_, s, st_);
      adj_solve(2, shift_);
      AdjPCGridArgs<T> g{};
      g.lsb_x = t1_;
      g.lsb_y = t1_ + pl;
      g.lam_jz = lam_jz_;
      g.jp_x = jp_[0];
      g.jp_y = jp_[1];
      g.lam_bx = lam_b_[0];
      g.lam_by = lam_b_[1];
      g.shift = shift_;
      g.inv2dz = 0.5 / cfg_.dzeta;
      launch_adj_pc_grid<T>(geom_, g, st_);
      pa.f = {t.f[1], t.f[2], t.f[3], tape_b(t, m, 0), tape_b(t, m, 1), t.f[4]};
      pa.lsb_x = t1_;
      pa.lsb_y = t1_ + pl;
      pa.lam_F[0] = lam_f_[0];
      pa.lam_F[1] = lam_f_[1];
      pa.lam_F[2] = lam_f_[2];
      pa.lam_F[3] = lam_b_[0];
      pa.lam_F[4] = lam_b_[1];
      pa.lam_F[5] = lam_f_[5];
      pa.acc = M > 1 ? lam_acc_ : nullptr;
      if (m > 0) {
        pa.acc_mode = m == M - 1 ? 1 : 2;
        launch_adj_trial_later<T>(geom_, lat_, pa, st_);
      } else {
        pa.acc_mode = 0;
        launch_adj_push<T>(geom_, lat_, pa, true, st_);
      }
      lbx = lam_b_[0];
      lby = lam_b_[1];
    }
    // initial guess B^0 = 2 B_{k-1} - B_{k-2}
    launch_adj_guess(pl, lbx, lby, carry_b2_[0], carry_b2_[1], carry_b1_[0], carry_b1_[1],
                     carry_b2_[0], carry_b2_[1], st_);
    // psi (with Ex-By = -d_x psi, Ey+Bx = -d_y psi), Ez and Bz solves
    {
      AdjSrcArgs<T> s{};
      s.count = 3;
      s.p0[0] = lam_psi_;
      s.p1[0] = lam_f_[0];
      s.p2[0] = lam_f_[1];
      s.c0[0] = s.c1[0] = s.c2[0] = 1.0;
      s.p0[1] = lam_f_[2];
      s.c0[1] = 1.0;
      s.p0[2] = lam_f_[5];
      s.c0[2] = 1.0;
      for (int q = 0; q < 3; ++q) s.out[q] = t2_ + q * pl;
      launch_adj_source<T>(geom_, s, st_);
      adj_solve(3, 0.0);
    }
    // adjoints of the deposit channels of slice k and the beam gradient
    {
      AdjDepGridArgs<T> d{};
      d.lpsi = t1_;
      d.lez = t1_ + pl;
      d.lbz = t1_ + 2 * pl;
      d.lam_jz = lam_jz_;
      d.carry_jx = carry_j_[0];
      d.carry_jy = carry_j_[1];
      d.lam_r = lam_psi_;
      d.lam_jx = carry_j_[0];
      d.lam_jy = carry_j_[1];
      d.bgx = bgx_;
      d.bgy = bgy_;
      d.dbgx = dbgx_;
      d.dbgy = dbgy_;
      d.grad_amp = grad_amp;
      d.grad_sigma = grad_sigma;
      d.amp = has_gauss_ ? amp_[k] : 0.0;
      d.k = k;
      launch_adj_dep_grid<T>(geom_, d, st_);
    }
    {
      AdjDepArgs<T> a{};
      a.p = t.p;
      a.lam_dep[0] = lam_psi_;
      a.lam_dep[1] = carry_j_[0];
      a.lam_dep[2] = carry_j_[1];
      a.lam_dep[3] = lam_jz_;
      a.lam_y = lam_y_;
      a.psi_floor = cfg_.psi_floor;
      launch_adj_deposit<T>(geom_, lat_, a, st_);
    }
    // the adjoint of J_perp_{k-1} collected here is slice k-1's carry
    std::swap(carry_j_[0], jp_[0]);
    std::swap(carry_j_[1], jp_[1]);
  }

  // Cells of LDS deposit histogram around a push tile: particles whose
  // stencil reaches further than this from their tile go to global atomics.
  // The wide stencils of orders 2 and 3 get one more cell.
  int default_tile_halo() const {
    int h = cfg_.shape_order >= 2 ? 3 : 2;
    if (const char* e = std::getenv("QSP_HALO")) {   // tuning override
      const int v = std::atoi(e);
      if (v >= 1 && v <= 16) h = v;
    }
    return h;
  }

  // Lattice rows per push workgroup (64 sites wide): as many rows as keep
  // >= min_wgs workgroups per launch, between 4 and 16.  The trial pushes and
  // the adjoint take 2048 (at 1024^2 sites 8 rows, 16 at 2048^2, 4 at 512^2),
  // the real push 4096 (at 1024^2 sites 4 rows: 72 against 75 us with 8 and
  // 86 with 16, while the trial pushes are faster with 8).
  int default_tile_rows(int64_t min_wgs = 2048) const {
    const int tx = lat_.nX < 64 ? lat_.nX : 64;
    int r = 16;
    while (r > 4 && r * tx > kBlock && lat_.np / (static_cast<int64_t>(tx) * r) < min_wgs) r >>= 1;
    if (const char* e = std::getenv("QSP_TILE_ROWS")) {   // tuning override
      const int v = std::atoi(e);
      if (v >= 1 && v <= 16 && (v & (v - 1)) == 0 && v * tx >= kBlock) r = v;
    }
    return r < lat_.nY ? r : lat_.nY;
  }
  size_t nodes() const { return static_cast<size_t>(cfg_.nx + 1) * (cfg_.ny + 1); }
  size_t elem_size(int q) const { return q < QSP_RHO_MJZ ? sizeof(T) : sizeof(double); }

  template <typename U>
  U* alloc(size_t n) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(n * sizeof(U), 256);
    const hipError_t e = hipMalloc(&p, bytes);
    if (e == hipErrorOutOfMemory) throw std::bad_alloc();
    QSP_HIP(e);
    allocs_.push_back(p);
    bytes_ += static_cast<int64_t>(bytes);
    return static_cast<U*>(p);
  }

  template <typename U>
  U* beam_alloc(size_t n) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(n * sizeof(U), 256);
    const hipError_t e = hipMalloc(&p, bytes);
    if (e == hipErrorOutOfMemory) throw std::bad_alloc();
    QSP_HIP(e);
    beam_allocs_.push_back(p);
    bytes_ += static_cast<int64_t>(bytes);
    beam_bytes_ += static_cast<int64_t>(bytes);
    return static_cast<U*>(p);
  }

  void free_beam() {
    (void)hipStreamSynchronize(st_);
    for (void* p : beam_allocs_) (void)hipFree(p);
    beam_allocs_.clear();
    bytes_ -= beam_bytes_;
    beam_bytes_ = 0;
    beam_n_ = 0;
    moving_beam_ = false;
    beam_soa_ = beam_tmp_ = nullptr;
    bs_ = BeamScratch{};
    beam_off_.clear();
  }

  void release() {
    (void)hipStreamSynchronize(st_);
    for (void* p : allocs_) (void)hipFree(p);
    allocs_.clear();
    if (ev0_) (void)hipEventDestroy(ev0_);
    if (ev1_) (void)hipEventDestroy(ev1_);
    ev0_ = ev1_ = nullptr;
  }

  void allocate() {
    const size_t pl = plane();
    psi_ = alloc<T>(pl);
    exmby_ = alloc<T>(pl);
    eypbx_ = alloc<T>(pl);
    ez_ = alloc<T>(pl);
    bz_ = alloc<T>(pl);
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 2; ++c) b_[b][c] = alloc<T>(pl);
    t1_ = alloc<T>(4 * pl);
    t2_ = alloc<T>(4 * pl);
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 5; ++c) dep_[d][c] = alloc<double>(pl);
    trial_[0] = alloc<double>(pl);
    trial_[1] = alloc<double>(pl);
    trial_sh_[0] = alloc<double>(pl);
    trial_sh_[1] = alloc<double>(pl);
    if (!explicit_) trial_rec_ = alloc<T>(6 * static_cast<size_t>(lat_.np));
    const size_t np = static_cast<size_t>(lat_.np);
    p_.xi_x = alloc<T>(np);
    p_.xi_y = alloc<T>(np);
    p_.ux = alloc<T>(np);
    p_.uy = alloc<T>(np);
    p_.psi = alloc<T>(np);
    p_.w = alloc<T>(np);
    p_.hist = alloc<T>(20 * np);
    p_.pab = alloc<T>(5 * np);
    twx_ = alloc<Cplx<T>>(2 * cfg_.nx);
    prex_ = alloc<T>(cfg_.nx);
    lamx_ = alloc<double>(cfg_.nx);
    twy_ = alloc<Cplx<T>>(2 * cfg_.ny);
    prey_ = alloc<T>(cfg_.ny);
    lamy_ = alloc<double>(cfg_.ny);
    bgx_ = alloc<double>(cfg_.nx + 1);
    bgy_ = alloc<double>(cfg_.ny + 1);
    dbgx_ = alloc<double>(cfg_.nx + 1);
    dbgy_ = alloc<double>(cfg_.ny + 1);
    if (explicit_) {
      for (int c = 0; c < 3; ++c) ex_dep_[c] = alloc<double>(pl);
      ex_x_ = alloc<double>(2 * pl);
      ex_r_ = alloc<double>(2 * pl);
      ex_q_ = alloc<double>(2 * pl);
      ex_p_[0] = alloc<double>(2 * pl);
      ex_p_[1] = alloc<double>(2 * pl);
      ex_partial_ = alloc<double>(static_cast<size_t>(explicit_partial_count(geom_)) * 9);
      ex_s_ = alloc<ExplicitScalars>(1);
    }
    if (cfg_.shape_order != 1) {
      ionx_ = alloc<double>(cfg_.nx + 1);
      iony_ = alloc<double>(cfg_.ny + 1);
    }
    iters_own_ = alloc<int32_t>(cfg_.nzeta);
    ctr_ = alloc<DevCounters>(1);
    partial_ = alloc<double>(2 * static_cast<size_t>(pc_partial_count(geom_)) + 2);
    if (cfg_.mem_cap_bytes > 0 && bytes_ > cfg_.mem_cap_bytes) throw std::bad_alloc();
  }

  // Per-axis tables of the sine transform (tw holds 2n entries, pre n):
  // the half-length transform's twiddles e^{-2 pi i m/n} and pre-twiddles
  // sin(pi m/n), or for the FP32 core of 256-1024 points the twiddles
  // W_2n^{l k1} at [k1 * 64 + l] and, in pre, the W_64^{la c1} table at
  // [la * 9 + c1] (complex); and the Laplacian eigenvalues.
  void axis_tables(int n, double h, Cplx<T>* tw, T* pre, double* lam) {
    std::vector<Cplx<T>> htw(2 * n);
    std::vector<T> hpre(n);
    std::vector<double> hlam(n);
    const double pi = 3.14159265358979323846;
    auto unit = [&](long q, long m) {   // e^{-2 pi i q / m}
      const double a = -2.0 * pi * static_cast<double>(q % m) / static_cast<double>(m);
      return Cplx<T>{static_cast<T>(std::cos(a)), static_cast<T>(std::sin(a))};
    };
    if (fast_core(sizeof(T), n)) {
      const int NL = core_lanes(sizeof(T), n), P = 2 * n / NL;
      for (int k1 = 0; k1 < P; ++k1)
        for (int l = 0; l < NL; ++l) htw[k1 * NL + l] = unit(static_cast<long>(l) * k1, 2 * n);
      Cplx<T>* w = reinterpret_cast<Cplx<T>*>(hpre.data());
      for (int i = 0; i < NL / 8 * 9; ++i) w[i] = Cplx<T>{T(0), T(0)};
      for (int la = 0; la < NL / 8; ++la)
        for (int c1 = 0; c1 < 8; ++c1) w[la * 9 + c1] = unit(la * c1, NL);
    } else {
      for (int m = 0; m < n; ++m) {
        htw[m] = unit(m, n);
        hpre[m] = static_cast<T>(std::sin(pi * m / n));
      }
    }
    for (int m = 0; m < n; ++m) {
      const double s = std::sin(pi * m / (2.0 * n));
      hlam[m] = -4.0 / (h * h) * s * s;
    }
    QSP_HIP(hipMemcpy(tw, htw.data(), 2 * n * sizeof(Cplx<T>), hipMemcpyHostToDevice));
    QSP_HIP(hipMemcpy(pre, hpre.data(), n * sizeof(T), hipMemcpyHostToDevice));
    QSP_HIP(hipMemcpy(lam, hlam.data(), n * sizeof(double), hipMemcpyHostToDevice));
  }

  void build_tables() {
    axis_tables(cfg_.nx, geom_.hx, twx_, prex_, lamx_);
    axis_tables(cfg_.ny, geom_.hy, twy_, prey_, lamy_);
    std::vector<double> z(std::max(cfg_.nx, cfg_.ny) + 1, 0.0);
    QSP_HIP(hipMemcpy(bgx_, z.data(), (cfg_.nx + 1) * sizeof(double), hipMemcpyHostToDevice));
    QSP_HIP(hipMemcpy(bgy_, z.data(), (cfg_.ny + 1) * sizeof(double), hipMemcpyHostToDevice));
    QSP_HIP(hipMemcpy(dbgx_, z.data(), (cfg_.nx + 1) * sizeof(double), hipMemcpyHostToDevice));
    QSP_HIP(hipMemcpy(dbgy_, z.data(), (cfg_.ny + 1) * sizeof(double), hipMemcpyHostToDevice));
    if (ionx_) {
      const std::vector<double> fx = ion_profile(cfg_.nx, cfg_.ppc_x, cfg_.shape_order);
      const std::vector<double> fy = ion_profile(cfg_.ny, cfg_.ppc_y, cfg_.shape_order);
      QSP_HIP(hipMemcpy(ionx_, fx.data(), fx.size() * sizeof(double), hipMemcpyHostToDevice));
      QSP_HIP(hipMemcpy(iony_, fy.data(), fy.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    QSP_HIP(hipMemset(ctr_, 0, sizeof(DevCounters)));
    if (ex_s_) QSP_HIP(hipMemset(ex_s_, 0, sizeof(ExplicitScalars)));
    QSP_HIP(hipDeviceSynchronize());
  }

  AxisTables<T> tx() const { return {twx_, prex_, lamx_}; }
  AxisTables<T> ty() const { return {twy_, prey_, lamy_}; }

  void zero_shared() {
    launch_zero(trial_sh_[0], plane(), st_);
    launch_zero(trial_sh_[1], plane(), st_);
  }

  void to_nodes_d(const double* src, double* dst) { launch_to_nodes<double>(geom_, src, dst, st_); }

  void add_out(OutCopy& oc, int q, void* dst, int kind) {
    if (oc.count >= kMaxOut) throw std::runtime_error("too many outputs");
    const int i = oc.count++;
    oc.dst[i] = dst;
    oc.kind[i] = kind;
    oc.is_double[i] = (q >= QSP_RHO_MJZ) || sizeof(T) == 8;
    oc.add_beam[i] = 0;
    oc.add_ion[i] = 0;
    oc.src2[i] = nullptr;
    double* const* dc = dep_[ic_];
    switch (q) {
      case QSP_PSI: oc.src[i] = psi_; break;
      case QSP_EXMBY: oc.src[i] = exmby_; break;
      case QSP_EYPBX: oc.src[i] = eypbx_; break;
      case QSP_EZ: oc.src[i] = ez_; break;
      case QSP_BX: oc.src[i] = b_[ik_][0]; break;
      case QSP_BY: oc.src[i] = b_[ik_][1]; break;
      case QSP_BZ: oc.src[i] = bz_; break;
      case QSP_RHO_MJZ: oc.src[i] = dc[0]; oc.add_ion[i] = 1; break;
      case QSP_JX: oc.src[i] = dc[1]; break;
      case QSP_JY: oc.src[i] = dc[2]; break;
      case QSP_JZ: oc.src[i] = dc[3]; oc.add_beam[i] = 1; break;
      case QSP_RHO:   // rho = (rho - Jz) + Jz, both FP64 sums
        oc.src[i] = dc[0]; oc.src2[i] = dc[3]; oc.add_beam[i] = 1; oc.add_ion[i] = 1; break;
      default: throw std::runtime_error("bad output id");
    }
  }

  SliceFields<T> fields(const T* bx, const T* by) const {
    return {exmby_, eypbx_, ez_, bx, by, bz_};
  }

  // one slice: the 2D slice routine followed by the real push to k+1
  void step(OutCopy& oc, int32_t* iters_out, double* resid_out) {
    const int k = cursor_;
    const double amp = has_gauss_ ? amp_[k] : 0.0;
    double* const* dp = dep_[ip_];
    double* const* dc = dep_[ic_];
    double* const* dn = dep_[in_];
    const size_t pl = plane();
    // the previous slice's real push deposited this slice's beam particles
    // unless the deposits are rebuilt here
    const bool beam_done = beam_ahead_ && dep_valid_;
    beam_ahead_ = false;
    if (!dep_valid_) {
      timed(QSP_K_OTHER, [&] {
        for (int c = 0; c < 5; ++c) launch_zero(dc[c], pl, st_);
        zero_shared();
      });
      PushArgs<T> a = push_args(fields(b_[ik_][0], b_[ik_][1]), dc, k);
      a.tile_rows = real_tile_rows_;
      timed(QSP_K_OTHER, [&] { launch_push<T>(geom_, lat_, a, kDepositOnly, ctr_, st_); });
      dep_valid_ = true;
    }
    T* bxk = b_[ik_][0];
    T* byk = b_[ik_][1];
    // the beam kernels of slice k read its particle range on the device; a
    // captured box launches them for every slice (the ranges change from
    // box to box), eager launches only where the slice holds particles
    const int64_t bcount = beam_n_ ? beam_off_[k + 1] - beam_off_[k] : 0;
    const bool beam_here = capturing_ ? beam_n_ > 0 : bcount > 0;
    const int64_t bgrid = capturing_ ? std::min<int64_t>(beam_n_, kBeamGraphThreads) : bcount;
    // beam deposit of slice k (Sec. II step 3)
    if (beam_here && !beam_done)
      timed(QSP_K_OTHER, [&] {
        launch_beam_deposit(geom_, beam_soa_, beam_n_, bs_.off, k, bgrid, cfg_.dzeta, dc[0], dc[3],
                            nullptr, st_);
      });
    // explicit beam current of slice k
    if (!cur_.empty() && cur_[k])
      timed(QSP_K_OTHER, [&] { launch_add_current(pl, cur_[k], dc[3], nullptr, st_); });
    // psi, Ez, Bz (Sec. II steps 4-6)
    {
      SrcPEZ<T> s{dc[0], dc[1], dc[2], cfg_.n0, ionx_, iony_, t1_};
      timed(QSP_K_ROW_FWD, [&] { launch_src_fwd_pez<T>(geom_, s, tx(), st_); });
      ColArgs<T> c{};
      c.in = t1_;
      c.out = t2_;
      c.out_dy = t2_ + 3 * pl;
      c.shift[0] = c.shift[1] = c.shift[2] = 0.0;
      c.honor_done = 0;
      c.w = col_width<T>(geom_, 3);
      // the deposit planes of slice k+1 are free: clear them for the real push
      for (int q = 0; q < 4; ++q) c.zero.p[q] = dn[q];
      c.zero.count = 4;
      if (explicit_)   // and the explicit solver's deposits for slice k
        for (int q = 0; q < 3; ++q) c.zero.p[c.zero.count++] = ex_dep_[q];
      c.zero.n = pl;
      timed(QSP_K_COL, [&] { launch_col_solve<T>(geom_, c, 3, ty(), lamx_, ctr_, st_); });
      RowInvArgs<T> r{};
      r.in[0] = t2_;
      r.out[0] = psi_;
      r.out_dx[0] = exmby_;
      r.in[1] = t2_ + 3 * pl;
      r.out[1] = eypbx_;
      r.in[2] = t2_ + pl;
      r.out[2] = ez_;
      r.in[3] = t2_ + 2 * pl;
      r.out[3] = bz_;
      r.in_strip = geom_.strip;
      // Bx/By initial guess of the predictor-corrector rides along
      r.guess = {bxk, byk, b_[i1_][0], b_[i1_][1], b_[i2_][0], b_[i2_][1], ctr_,
                 tape_slot_ ? tape_b(*tape_slot_, 0, 0) : nullptr,
                 tape_slot_ ? tape_b(*tape_slot_, 0, 1) : nullptr};
      timed(QSP_K_ROW_INV, [&] { launch_row_inv<T>(geom_, r, 4, tx(), st_); });
      dst_solves_ += 3;
    }
    // predictor-corrector iterations launched for this slice
    const int pc_launch = budget_on_ ? budget_launch_[k] : cfg_.pc_max_iter;
    const int budgeted = pc_launch < cfg_.pc_max_iter ? 1 : 0;
    // Bx/By (Sec. II step 7, Sec. III.B): explicit solver or predictor-corrector
    if (explicit_) {
      explicit_bxby(k, dc, amp, bxk, byk);
    } else {
      {
        PushArgs<T> a = push_args(fields(bxk, byk), trial_, k, 2, trial_sh_);
        // taped slices keep their record for the reverse pass
        a.rec = tape_slot_ ? tape_slot_->rec : trial_rec_;
        // a slot's particle arrays are one block of 26 planes (alloc_particles)
        if (tape_slot_) a.tape = tape_slot_->p.xi_x;
        const PushMode first_trial = tape_slot_ ? kPushTrialTape : kPushTrial;
        a.pc_partial = partial_;
        a.pc_nblk = pc_partial_count(geom_);
        SrcBxBy<T> s{};
        s.jz = dc[3];
        s.jx_prev = dp[1];
        s.jy_prev = dp[2];
        s.jx_next = trial_[0];
        s.jy_next = trial_[1];
        s.sx_next = trial_sh_[0];
        s.sy_next = trial_sh_[1];
        s.bx = bxk;
        s.by = byk;
        s.shift = shift_;
        s.dzeta = cfg_.dzeta;
        s.beam_amp = amp;
        s.bgx = bgx_;
        s.bgy = bgy_;
        s.out = t1_;
        ColArgs<T> c{};
        c.in = t1_;
        c.out = t2_;
        c.out_dy = nullptr;
        c.shift[0] = c.shift[1] = shift_;
        c.honor_done = 1;
        c.w = col_width<T>(geom_, 2);
        // the trial currents have been read: clear what the next trial adds
        // into (the shared planes; with no tiles the owner planes)
        c.zero.p[0] = tiled_ ? trial_sh_[0] : trial_[0];
        c.zero.p[1] = tiled_ ? trial_sh_[1] : trial_[1];
        c.zero.count = 2;
        c.zero.n = pl;
        for (int m = 0; m < pc_launch; ++m) {
          a.pc_iter = m;
          // the first trial push of the slice leaves the record the later
          // ones start from (and on a taped slice the slice-k particle state)
          const PushMode tm = m == 0 ? first_trial : kTrialLater;
          timed(QSP_K_TRIAL, [&] { launch_push<T>(geom_, lat_, a, tm, ctr_, st_); });
          timed(QSP_K_ROW_FWD, [&] { launch_src_fwd_bxby<T>(geom_, s, tx(), ctr_, st_); });
          timed(QSP_K_COL, [&] { launch_col_solve<T>(geom_, c, 2, ty(), lamx_, ctr_, st_); });
          PCArgs<T> pc{t2_, bxk, byk, partial_, cfg_.pc_tol,
                       tape_slot_ ? tape_b(*tape_slot_, m + 1, 0) : nullptr,
                       tape_slot_ ? tape_b(*tape_slot_, m + 1, 1) : nullptr};
          timed(QSP_K_ROW_INV, [&] { launch_row_inv_pc<T>(geom_, pc, tx(), ctr_, st_); });
        }
      }
    }
    // beam particles of slice k take their time step in the final fields
    // (with the real push below when there is one)
    const bool beam_push_here = beam_here && beam_dt_ != 0.0;
    if (beam_push_here && k + 1 >= cfg_.nzeta) {
      timed(QSP_K_OTHER, [&] {
        launch_beam_push<T>(geom_, beam_soa_, beam_n_, bs_.off, k, bgrid, fields(bxk, byk), beam_dt_,
                            st_);
      });
      beam_dirty_ = true;
    }
    // outputs of slice k
    oc.beam_amp = amp;
    oc.n0 = cfg_.n0;
    oc.ionx = ionx_;
    oc.iony = iony_;
    oc.bgx = bgx_;
    oc.bgy = bgy_;
    if (oc.count) timed(QSP_K_OTHER, [&] { launch_out_copy(geom_, oc, st_); });
    // real push to slice k+1 with deposit there (Sec. II step 1 of the next
    // slice); it also closes the predictor-corrector bookkeeping of slice k
    if (k + 1 < cfg_.nzeta) {
      PushArgs<T> a = push_args(fields(bxk, byk), dn, k);
      a.tile_rows = real_tile_rows_;
      if (!explicit_) {   // the last corrector solve's convergence test
        a.pc_partial = partial_;
        a.pc_nblk = pc_partial_count(geom_);
      }
      a.iters_out = iters_out;
      a.iters_own = iters_own_ + k;
      a.resid_out = resid_out;
      a.pc_budgeted = budgeted;
      if (beam_n_ > 0) {
        // the launch also pushes slice k's beam particles and deposits
        // slice k+1's (into the planes it deposits the plasma into)
        const int64_t ncount = beam_off_[k + 2] - beam_off_[k + 1];
        const int64_t ngrid = capturing_ ? std::min<int64_t>(beam_n_, kBeamGraphThreads) : ncount;
        const auto wgs = [](int64_t c) {
          return static_cast<int>(std::min<int64_t>((c + kBlock - 1) / kBlock, 1024));
        };
        a.beam = {beam_soa_, beam_n_, bs_.off, beam_dt_, beam_push_here ? wgs(bgrid) : 0,
                  (capturing_ || ncount > 0) ? wgs(ngrid) : 0};
        if (beam_push_here) beam_dirty_ = true;
        beam_ahead_ = true;
      }
      const auto job = [this, a] { launch_push<T>(geom_, lat_, a, kPushReal, ctr_, st_); };
      if (capturing_ && timer_.active(cursor_)) {
        // the sampled launch runs between graph segments, under its events
        end_segment();
        cap_graph_->items.push_back({nullptr, std::function<void()>(job), QSP_K_PUSH});
        begin_segment();
      } else {
        timed(QSP_K_PUSH, job);
      }
      pushes_ += lat_.np;
    } else {
      timed(QSP_K_OTHER, [&] {
        launch_slice_end(ctr_, iters_out, iters_own_ + k, resid_out, cfg_.pc_tol, cfg_.pc_max_iter,
                         budgeted,
                         explicit_ ? nullptr : partial_, pc_partial_count(geom_), st_);
      });
    }
    // hand-off: J_perp of k becomes the previous slice's, B rotates
    const int old_p = ip_;
    ip_ = ic_;
    ic_ = in_;
    in_ = old_p;
    const int old2 = i2_;
    i2_ = i1_;
    i1_ = ik_;
    ik_ = old2;
    ++cursor_;
    ++slices_done_;
  }

  // Explicit Bx/By solver of slice k (Sec. III.B): deposit chi, DJx, DJy
  // from the slice-k plasma in the final psi, Ez, Bz, then solve
  // (lap - chi) B = R by preconditioned conjugate gradients, starting from
  // the guess 2 B_{k-1} - B_{k-2} already in bxk, byk; at most pc_max_iter
  // iterations, relative residual target pc_tol.
  void explicit_bxby(int k, double* const* dc, double amp, T* bxk, T* byk) {
    const size_t pl = plane();
    PushArgs<T> d = push_args(fields(bxk, byk), ex_dep_, k, 3);
    timed(QSP_K_TRIAL, [&] { launch_push<T>(geom_, lat_, d, kExplicitDep, ctr_, st_); });
    ExplicitArgs<T> a{};
    a.jz = dc[3];
    a.beam_amp = amp;
    a.bgx = bgx_;
    a.bgy = bgy_;
    a.chi = ex_dep_[0];
    a.djx = ex_dep_[1];
    a.djy = ex_dep_[2];
    a.b[0] = bxk;
    a.b[1] = byk;
    a.x = ex_x_;
    a.r = ex_r_;
    a.q = ex_q_;
    a.p[0] = ex_p_[0];
    a.p[1] = ex_p_[1];
    a.fwd = t1_;
    a.col = t2_;
    a.z = t1_ + 2 * pl;
    const size_t np = static_cast<size_t>(explicit_partial_count(geom_));
    a.part_s = ex_partial_;
    a.part_z = ex_partial_ + 2 * np;
    a.part_m = ex_partial_ + 6 * np;
    a.part_u = ex_partial_ + 8 * np;
    a.s = ex_s_;
    a.tol = cfg_.pc_tol;
    // the solver's planes between its row and column passes stay row-major
    Geom ge = geom_;
    ge.strip = 0;
    ColArgs<T> c{};
    c.in = t1_;
    c.out = t2_;
    c.out_dy = nullptr;
    c.shift[0] = c.shift[1] = shift_;
    c.honor_done = 1;
    c.w = col_width<T>(ge, 2);
    auto precondition = [&](int it) {
      a.it = it;
      timed(QSP_K_COL, [&] { launch_col_solve<T>(ge, c, 2, ty(), lamx_, ctr_, st_); });
      timed(QSP_K_ROW_INV, [&] { launch_explicit<T>(ge, a, kExplRowInv, tx(), ctr_, st_); });
    };
    a.it = 0;
    timed(QSP_K_ROW_FWD, [&] { launch_explicit<T>(ge, a, kExplSetup, tx(), ctr_, st_); });
    precondition(0);
    for (int m = 1; m <= cfg_.pc_max_iter; ++m) {
      a.it = m;
      timed(QSP_K_OTHER, [&] { launch_explicit<T>(ge, a, kExplMatvec, tx(), ctr_, st_); });
      timed(QSP_K_ROW_FWD, [&] { launch_explicit<T>(ge, a, kExplUpdate, tx(), ctr_, st_); });
      if (m < cfg_.pc_max_iter) precondition(m);
    }
    a.it = cfg_.pc_max_iter;
    timed(QSP_K_OTHER, [&] { launch_explicit<T>(ge, a, kExplClose, tx(), ctr_, st_); });
    dst_solves_ += 2 * (cfg_.pc_max_iter);
  }

  PushArgs<T> push_args(const SliceFields<T>& f, double* const* ch, int k, int nch = 4,
                        double* const* sh = nullptr) {
    PushArgs<T> a{};
    a.p = p_;
    a.f = f;
    for (int c = 0; c < nch; ++c) {
      a.dep.ch[c] = ch[c];
      a.dep.sh[c] = sh ? sh[c] : nullptr;
    }
    a.k = k;
    a.dzeta = cfg_.dzeta;
    a.hx = geom_.hx;
    a.hy = geom_.hy;
    a.psi_floor = cfg_.psi_floor;
    a.tiled = tiled_ ? 1 : 0;
    a.tile_rows = tile_rows_;
    a.tile_halo = tile_halo_;
    a.pc_tol = cfg_.pc_tol;
    a.pc_max_iter = cfg_.pc_max_iter;
    return a;
  }

  // brackets one launch with timer events when slice k is sampled; while a
  // box is captured into graphs there are no events
  template <typename F>
  void timed(int cls, F&& launch) {
    if (capturing_) {
      launch();
      return;
    }
    const bool on = timer_.active(cursor_);
    if (on) timer_.begin(cls, st_);
    launch();
    if (on) timer_.end(st_);
  }

  hipStream_t st_;
  int device_;
  KernelTimer timer_;
  // macro-particle beam (sorted by slice)
  std::vector<void*> beam_allocs_;
  int64_t beam_bytes_ = 0;
  float* beam_soa_ = nullptr;
  float* beam_tmp_ = nullptr;
  int64_t beam_n_ = 0;
  double beam_dt_ = 0.0;
  bool beam_dirty_ = false;
  bool beam_ahead_ = false;   // slice cursor_'s beam deposit is already done
  BeamScratch bs_{};
  std::vector<int64_t> beam_off_;
  std::vector<double*> cur_;          // explicit beam current per slice (or null)
  std::vector<void*> allocs_;
  int64_t bytes_ = 0;
  T *psi_ = nullptr, *exmby_ = nullptr, *eypbx_ = nullptr, *ez_ = nullptr, *bz_ = nullptr;
  T* b_[3][2] = {};
  T *t1_ = nullptr, *t2_ = nullptr;
  double* dep_[3][5] = {};
  double* trial_[2] = {};
  // shared deposit planes of the trial pushes (DepOut::sh), cleared by each
  // predictor-corrector iteration's column pass
  double* trial_sh_[2] = {};
  T* trial_rec_ = nullptr;   // record of the slice's first trial push
  Particles<T> p_{};
  Cplx<T>* twx_ = nullptr;
  Cplx<T>* twy_ = nullptr;
  T *prex_ = nullptr, *prey_ = nullptr;
  double *lamx_ = nullptr, *lamy_ = nullptr, *bgx_ = nullptr, *bgy_ = nullptr;
  double *dbgx_ = nullptr, *dbgy_ = nullptr;
  double *ionx_ = nullptr, *iony_ = nullptr;   // ion profile factors, null for order 1
  // adjoint: checkpoints, tape of one chunk, reverse work space
  std::vector<void*> adj_allocs_;
  int64_t adj_bytes_ = 0;
  std::pair<int, int> adj_shape_{0, 0};
  std::vector<Checkpoint<T>> ckpt_;
  std::vector<TapeSlot<T>> tape_;
  TapeSlot<T>* tape_slot_ = nullptr;
  int rec_K_ = 1;
  int32_t* iters_dev_ = nullptr;
  std::vector<int32_t> iters_host_;
  T *lam_y_ = nullptr, *lam_ring_ = nullptr;
  T* lam_acc_ = nullptr;   // later P-C iterations' adjoint sums [7][np]
  double* lam_f_[6] = {};
  double *lam_psi_ = nullptr, *lam_jz_ = nullptr;
  double* jp_[2] = {};
  double* carry_j_[2] = {};
  double* carry_b1_[2] = {};
  double* carry_b2_[2] = {};
  double* lam_b_[2] = {};
  DevCounters* ctr_ = nullptr;
  double* partial_ = nullptr;
  std::vector<double> amp_;
  double shift_ = 0.0;
  bool explicit_ = false;
  bool graphs_ = true;            // replay whole boxes from HIP graphs
  bool capturing_ = false;
  hipStream_t cap_st_ = nullptr;  // capture stream
  uint64_t launch_version_ = 0;
  // speculative P-C launch budgets (run_box_graphs)
  int32_t* iters_own_ = nullptr;   // per-slice iteration counts of the last box
  std::vector<int> budget_;          // learned: iterations the slices needed so far
  std::vector<int> budget_launch_;   // launched in the speculative box
  std::vector<int> margin_;          // 1: the slice's count has risen before
  bool budget_ready_ = false;
  uint64_t budget_version_ = 0;    // launch_version_ the budgets were learned under
  bool budget_on_ = false;         // step() launches budget_[k] iterations
  int spec_mode_ = 1;
  bool fresh_box_ = false;         // plasma as init_plasma left it, cursor 0
  int64_t box_reruns_ = 0;
  BoxGraph graph_;     // every slice launches pc_max_iter P-C iterations
  BoxGraph graph_b_;   // launches as many as the budgets hold
  BoxGraph* cap_graph_ = nullptr;   // the graph being captured
  // explicit Bx/By solver: deposits chi, DJx, DJy and the Krylov vectors
  double* ex_dep_[3] = {nullptr, nullptr, nullptr};
  double *ex_x_ = nullptr, *ex_r_ = nullptr, *ex_q_ = nullptr;
  double* ex_p_[2] = {nullptr, nullptr};
  double* ex_partial_ = nullptr;
  ExplicitScalars* ex_s_ = nullptr;
  int ip_ = 0, ic_ = 1, in_ = 2;   // deposit buffers of slices k-1, k, k+1
  int ik_ = 0, i1_ = 1, i2_ = 2;   // B buffers of slices k, k-1, k-2
  bool dep_valid_ = false;
  bool tiled_ = true;
  int tile_rows_ = 16;
  int real_tile_rows_ = 16;   // of the real push and the deposit-only pass
  int tile_halo_ = 2;
  bool nonfinite_ = false;
  hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
  double last_ms_ = 0.0;
  int64_t slices_done_ = 0, dst_solves_ = 0, pushes_ = 0;
};

std::unique_ptr<BoxBase> make_box(const qsp_config& cfg, int device, hipStream_t stream) {
  if (cfg.precision == QSP_FP64) return std::make_unique<Box<double>>(cfg, device, stream);
  return std::make_unique<Box<float>>(cfg, device, stream);
}

}  // namespace qsp
