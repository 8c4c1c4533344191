// Host runtime of libqsp: one simulation box on one GPU.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "../../include/qsp.h"
#include "common.hpp"
#include "kernels.hpp"

namespace qsp {

// Host-side check of a configuration; returns an empty string when valid.
std::string validate(const qsp_config& c);

// Default screening shift of the predictor-corrector iteration: the linear
// response of the centred d_zeta J_perp term to a change of Bx/By through one
// trial Adams-Bashforth step, (AB5_0 / 2) * n0.
double default_pc_shift(double n0);

// Ion density of the rest lattice along one axis (nodes 0..n) in units of
// n0, for the given particles per cell and shape order.
std::vector<double> ion_profile(int n, int ppc, int order);

class BoxBase {
 public:
  virtual ~BoxBase() = default;
  virtual void init_plasma() = 0;
  virtual void set_beam_gaussian(const double* amp, double sx, double sy, double x0,
                                 double y0) = 0;
  virtual void advance_slice(const qsp_slice_out* out) = 0;
  virtual void run_box(const qsp_box_out* out) = 0;
  virtual void get_stats(qsp_stats* s) = 0;
  virtual void get_state(qsp_slice_state* dst) = 0;
  virtual void set_state(const qsp_slice_state* src) = 0;
  virtual void set_deposit_tiled(bool on) = 0;
  virtual void set_beam_particles(int64_t n, const float* soa, double dt) = 0;
  // explicit Jz (= rho) of slice k, node layout FP64 on the device; NULL removes it
  virtual void set_beam_current(int k, const double* jz) = 0;
  virtual void clear_beam_currents() = 0;
  virtual void get_beam_particles(float* soa) = 0;
  virtual int64_t beam_count() const = 0;
  virtual void solve_poisson(int nbatch, const void* src, void* dst, double shift) = 0;
  virtual void set_timing(int every) = 0;
  virtual void get_kernel_times(qsp_kernel_times* out) = 0;
  // synchronises; true if a non-finite residual or norm was met
  virtual bool check_nonfinite() = 0;
  // checkpointed forward of slices 0 .. n_slices-1 and its reverse pass
  virtual void record(int n_slices, int ckpt_every, const qsp_box_out* out) = 0;
  virtual void adjoint(const qsp_box_cotangent* cot, double* grad_amp, double* grad_sigma,
                       double* loss) = 0;
  virtual int64_t adjoint_bytes(int n_slices, int ckpt_every) const = 0;
  bool recorded() const { return rec_valid_; }
  int recorded_slices() const { return rec_slices_; }
  bool has_gaussian_beam() const { return has_gauss_; }
  bool has_moving_beam() const { return moving_beam_; }
  int cursor() const { return cursor_; }
  bool initialised() const { return initialised_; }
  int64_t n_particles() const { return lat_.np; }
  const qsp_config& config() const { return cfg_; }

 protected:
  qsp_config cfg_{};
  Geom geom_{};
  Lattice lat_{};
  int cursor_ = 0;
  bool initialised_ = false;
  bool rec_valid_ = false;
  int rec_slices_ = 0;
  bool has_gauss_ = false;
  bool moving_beam_ = false;
};

std::unique_ptr<BoxBase> make_box(const qsp_config& cfg, int device, hipStream_t stream);

// bytes a context of this configuration will hold on the device
int64_t device_bytes_needed(const qsp_config& cfg);

// qsp_solve_poisson_noalloc (static scratch, no allocation); err holds the
// reason of a failure
qsp_status solve_poisson_noalloc(const qsp_config* cfg, int device, void* stream, int nbatch,
                                 const void* src, void* dst, double shift, std::string& err);

}  // namespace qsp
