// extern "C" entry points of libqsp (declared in include/qsp.h): argument and
// state checks, error translation and the sticky device-error state.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "runtime.hpp"

struct qsp_ctx_s {
  std::unique_ptr<qsp::BoxBase> box;
  std::string last_error;
  bool device_failed = false;
  bool beam_set = false;
  int device = 0;
};

namespace {

thread_local std::string g_last_error;

qsp_status fail(qsp_ctx ctx, qsp_status s, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  else g_last_error = msg;
  return s;
}

// Runs `body` with the context's device errors translated to status codes.
template <typename F>
qsp_status guarded(qsp_ctx ctx, F&& body) {
  if (!ctx) return fail(nullptr, QSP_ERR_INVALID_ARG, "null context");
  if (ctx->device_failed)
    return fail(ctx, QSP_ERR_DEVICE, "context is in the failed state after an earlier device error: " +
                                         ctx->last_error);
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(ctx, QSP_ERR_OUT_OF_MEMORY, "device or host allocation failed");
  } catch (const qsp::DeviceError& e) {
    ctx->device_failed = true;
    return fail(ctx, QSP_ERR_DEVICE, e.what());
  } catch (const std::exception& e) {
    ctx->device_failed = true;
    return fail(ctx, QSP_ERR_DEVICE, e.what());
  }
}

}  // namespace

extern "C" {

qsp_status qsp_validate_config(const qsp_config* cfg, char* msg, size_t msg_len) {
  std::string err = cfg ? qsp::validate(*cfg) : std::string("null config");
  if (msg && msg_len > 0) {
    std::strncpy(msg, err.c_str(), msg_len - 1);
    msg[msg_len - 1] = '\0';
  }
  if (!err.empty()) {
    g_last_error = err;
    return QSP_ERR_INVALID_ARG;
  }
  return QSP_OK;
}

qsp_status qsp_create(const qsp_config* cfg, int device, void* hip_stream, qsp_ctx* out) {
  if (!out) return fail(nullptr, QSP_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (!cfg) return fail(nullptr, QSP_ERR_INVALID_ARG, "null config");
  const std::string err = qsp::validate(*cfg);
  if (!err.empty()) return fail(nullptr, QSP_ERR_INVALID_ARG, err);
  if (cfg->mem_cap_bytes > 0 && qsp::device_bytes_needed(*cfg) > cfg->mem_cap_bytes)
    return fail(nullptr, QSP_ERR_OUT_OF_MEMORY,
                "configuration needs " + std::to_string(qsp::device_bytes_needed(*cfg)) +
                    " device bytes, above mem_cap_bytes");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(nullptr, QSP_ERR_INVALID_ARG, "no such HIP device");
  auto* ctx = new (std::nothrow) qsp_ctx_s();
  if (!ctx) return fail(nullptr, QSP_ERR_OUT_OF_MEMORY, "host allocation failed");
  ctx->device = device;
  try {
    ctx->box = qsp::make_box(*cfg, device, static_cast<hipStream_t>(hip_stream));
  } catch (const std::bad_alloc&) {
    delete ctx;
    return fail(nullptr, QSP_ERR_OUT_OF_MEMORY, "device allocation failed");
  } catch (const std::exception& e) {
    delete ctx;
    return fail(nullptr, QSP_ERR_DEVICE, e.what());
  }
  *out = ctx;
  return QSP_OK;
}

qsp_status qsp_destroy(qsp_ctx ctx) {
  if (!ctx) return QSP_OK;
  try {
    ctx->box.reset();
  } catch (...) {
  }
  delete ctx;
  return QSP_OK;
}

qsp_status qsp_init_plasma(qsp_ctx ctx) {
  return guarded(ctx, [&] {
    ctx->box->init_plasma();
    return QSP_OK;
  });
}

qsp_status qsp_set_beam_gaussian(qsp_ctx ctx, const double* amp, double sx, double sy,
                                 double x0, double y0) {
  return guarded(ctx, [&] {
    if (!amp) return fail(ctx, QSP_ERR_INVALID_ARG, "null amplitude array");
    const int nz = ctx->box->config().nzeta;
    for (int k = 0; k < nz; ++k)
      if (!std::isfinite(amp[k])) return fail(ctx, QSP_ERR_INVALID_ARG, "non-finite beam amplitude");
    if (!(sx > 0) || !(sy > 0) || !std::isfinite(sx) || !std::isfinite(sy))
      return fail(ctx, QSP_ERR_INVALID_ARG, "beam sigmas must be finite and > 0");
    if (!std::isfinite(x0) || !std::isfinite(y0))
      return fail(ctx, QSP_ERR_INVALID_ARG, "beam centre must be finite");
    ctx->box->set_beam_gaussian(amp, sx, sy, x0, y0);
    ctx->beam_set = true;
    return QSP_OK;
  });
}

qsp_status qsp_set_beam_particles(qsp_ctx ctx, int64_t n, const float* soa, double dt) {
  return guarded(ctx, [&] {
    if (n < 0 || n > 2147483647LL) return fail(ctx, QSP_ERR_INVALID_ARG, "n must be in [0, 2^31)");
    if (n > 0 && !soa) return fail(ctx, QSP_ERR_INVALID_ARG, "null particle array");
    if (!std::isfinite(dt)) return fail(ctx, QSP_ERR_INVALID_ARG, "dt must be finite");
    if (n > 0 && ctx->box->config().nzeta + 1 > qsp::kMaxBeamKeys)
      return fail(ctx, QSP_ERR_INVALID_ARG, "particle beams need nzeta < 16384");
    ctx->box->set_beam_particles(n, soa, dt);
    return QSP_OK;
  });
}

qsp_status qsp_get_beam_particles(qsp_ctx ctx, int64_t n, float* soa) {
  return guarded(ctx, [&] {
    if (ctx->box->beam_count() == 0) return fail(ctx, QSP_ERR_BAD_STATE, "no particle beam");
    if (n != ctx->box->beam_count())
      return fail(ctx, QSP_ERR_INVALID_ARG, "n does not match the stored particle count");
    if (!soa) return fail(ctx, QSP_ERR_INVALID_ARG, "null particle array");
    ctx->box->get_beam_particles(soa);
    return QSP_OK;
  });
}

qsp_status qsp_get_beam_count(qsp_ctx ctx, int64_t* n) {
  return guarded(ctx, [&] {
    if (!n) return fail(ctx, QSP_ERR_INVALID_ARG, "null output");
    *n = ctx->box->beam_count();
    return QSP_OK;
  });
}

qsp_status qsp_advance_slice(qsp_ctx ctx, const qsp_slice_out* out) {
  return guarded(ctx, [&] {
    if (!ctx->box->initialised()) return fail(ctx, QSP_ERR_BAD_STATE, "plasma not initialised");
    if (ctx->box->cursor() >= ctx->box->config().nzeta)
      return fail(ctx, QSP_ERR_BAD_STATE, "box already complete");
    ctx->box->advance_slice(out);
    return QSP_OK;
  });
}

qsp_status qsp_set_beam_current(qsp_ctx ctx, int32_t k, const double* jz) {
  return guarded(ctx, [&] {
    if (k == -1 && !jz) {
      ctx->box->clear_beam_currents();
      return QSP_OK;
    }
    if (k < 0 || k >= ctx->box->config().nzeta)
      return fail(ctx, QSP_ERR_INVALID_ARG, "slice index outside [0, nzeta)");
    ctx->box->set_beam_current(k, jz);
    return QSP_OK;
  });
}

qsp_status qsp_run_box(qsp_ctx ctx, const qsp_box_out* out, qsp_stats* stats) {
  return guarded(ctx, [&] {
    if (!ctx->box->initialised()) return fail(ctx, QSP_ERR_BAD_STATE, "plasma not initialised");
    if (ctx->box->cursor() >= ctx->box->config().nzeta)
      return fail(ctx, QSP_ERR_BAD_STATE, "box already complete");
    if (out && out->stack_every < 0) return fail(ctx, QSP_ERR_INVALID_ARG, "stack_every < 0");
    ctx->box->run_box(out);
    if (stats) ctx->box->get_stats(stats);
    if (ctx->box->check_nonfinite())
      return fail(ctx, QSP_ERR_NONFINITE, "non-finite predictor-corrector residual");
    return QSP_OK;
  });
}

qsp_status qsp_run_box_record(qsp_ctx ctx, int32_t n_slices, int32_t ckpt_every,
                              const qsp_box_out* out, qsp_stats* stats) {
  return guarded(ctx, [&] {
    const qsp::BoxBase& b = *ctx->box;
    if (!b.initialised() || b.cursor() != 0)
      return fail(ctx, QSP_ERR_BAD_STATE, "record needs the plasma initialised at slice 0");
    if (n_slices < 1 || n_slices > b.config().nzeta)
      return fail(ctx, QSP_ERR_INVALID_ARG, "n_slices must be in [1, nzeta]");
    if (ckpt_every < 1) return fail(ctx, QSP_ERR_INVALID_ARG, "ckpt_every must be >= 1");
    if (out && out->stack_every < 0) return fail(ctx, QSP_ERR_INVALID_ARG, "stack_every < 0");
    if (!b.has_gaussian_beam())
      return fail(ctx, QSP_ERR_BAD_STATE, "the adjoint needs a Gaussian beam (qsp_set_beam_gaussian)");
    if (b.has_moving_beam())
      return fail(ctx, QSP_ERR_BAD_STATE, "the adjoint does not transpose a moving particle beam");
    const qsp_config& c = b.config();
    if (c.shape_order < 1)
      return fail(ctx, QSP_ERR_INVALID_ARG, "the adjoint needs a shape order of 1, 2 or 3");
    if (c.bxby_solver != QSP_BXBY_PC)
      return fail(ctx, QSP_ERR_INVALID_ARG, "the adjoint transposes the predictor-corrector only");
    if (c.mem_cap_bytes > 0 && qsp::device_bytes_needed(c) + b.adjoint_bytes(n_slices, ckpt_every) >
                                   c.mem_cap_bytes)
      return fail(ctx, QSP_ERR_OUT_OF_MEMORY, "checkpoints and tape exceed mem_cap_bytes");
    ctx->box->record(n_slices, ckpt_every, out);
    if (stats) ctx->box->get_stats(stats);
    if (ctx->box->check_nonfinite())
      return fail(ctx, QSP_ERR_NONFINITE, "non-finite predictor-corrector residual");
    return QSP_OK;
  });
}

qsp_status qsp_run_box_adjoint(qsp_ctx ctx, const qsp_box_cotangent* cot, double* grad_amp,
                               double* grad_sigma, double* loss) {
  return guarded(ctx, [&] {
    if (!ctx->box->recorded())
      return fail(ctx, QSP_ERR_BAD_STATE, "no recorded forward pass (qsp_run_box_record)");
    if (!cot || !grad_amp || !grad_sigma)
      return fail(ctx, QSP_ERR_INVALID_ARG, "null cotangent or gradient output");
    if (cot->k_lo < 0 || cot->k_lo >= ctx->box->recorded_slices())
      return fail(ctx, QSP_ERR_INVALID_ARG, "k_lo outside the recorded slices");
    ctx->box->adjoint(cot, grad_amp, grad_sigma, loss);
    return QSP_OK;
  });
}

qsp_status qsp_get_stats(qsp_ctx ctx, qsp_stats* stats) {
  return guarded(ctx, [&] {
    if (!stats) return fail(ctx, QSP_ERR_INVALID_ARG, "null stats");
    ctx->box->get_stats(stats);
    return QSP_OK;
  });
}

static bool state_ptrs_ok(const qsp_slice_state* s) {
  return s && s->x && s->y && s->ux && s->uy && s->psi && s->w && s->hist && s->jx_prev &&
         s->jy_prev && s->bx_prev1 && s->by_prev1 && s->bx_prev2 && s->by_prev2;
}

qsp_status qsp_get_slice_state(qsp_ctx ctx, qsp_slice_state* dst) {
  return guarded(ctx, [&] {
    if (!state_ptrs_ok(dst)) return fail(ctx, QSP_ERR_INVALID_ARG, "null state pointer");
    if (dst->np != ctx->box->n_particles())
      return fail(ctx, QSP_ERR_INVALID_ARG, "np does not match the particle count");
    if (!ctx->box->initialised()) return fail(ctx, QSP_ERR_BAD_STATE, "plasma not initialised");
    ctx->box->get_state(dst);
    return QSP_OK;
  });
}

qsp_status qsp_set_slice_state(qsp_ctx ctx, const qsp_slice_state* src) {
  return guarded(ctx, [&] {
    if (!state_ptrs_ok(src)) return fail(ctx, QSP_ERR_INVALID_ARG, "null state pointer");
    const qsp_config& c = ctx->box->config();
    if (src->np != ctx->box->n_particles())
      return fail(ctx, QSP_ERR_INVALID_ARG, "np does not match the particle count");
    if (src->k < 0 || src->k >= c.nzeta) return fail(ctx, QSP_ERR_INVALID_ARG, "k out of range");
    for (int64_t i = 0; i < src->np; ++i) {
      if (src->w[i] != 0.0 &&
          !(src->x[i] >= c.x_lo && src->x[i] <= c.x_hi && src->y[i] >= c.y_lo && src->y[i] <= c.y_hi))
        return fail(ctx, QSP_ERR_INVALID_ARG, "particle outside the box");
      if (!std::isfinite(src->ux[i]) || !std::isfinite(src->uy[i]) || !std::isfinite(src->psi[i]) ||
          !std::isfinite(src->w[i]) || src->w[i] < 0)
        return fail(ctx, QSP_ERR_INVALID_ARG, "non-finite particle state");
    }
    ctx->box->set_state(src);
    return QSP_OK;
  });
}

qsp_status qsp_solve_poisson(qsp_ctx ctx, int32_t nbatch, const void* src, void* dst,
                             double shift) {
  return guarded(ctx, [&] {
    if (nbatch < 1 || nbatch > 4) return fail(ctx, QSP_ERR_INVALID_ARG, "nbatch must be in [1, 4]");
    if (!src || !dst) return fail(ctx, QSP_ERR_INVALID_ARG, "null array");
    if (!std::isfinite(shift) || shift < 0) return fail(ctx, QSP_ERR_INVALID_ARG, "shift must be finite and >= 0");
    ctx->box->solve_poisson(nbatch, src, dst, shift);
    return QSP_OK;
  });
}

qsp_status qsp_solve_poisson_noalloc(const qsp_config* cfg, int device, void* hip_stream,
                                     int32_t nbatch, const void* src, void* dst,
                                     double shift) {
  std::string err;
  const qsp_status st =
      qsp::solve_poisson_noalloc(cfg, device, hip_stream, nbatch, src, dst, shift, err);
  if (st != QSP_OK) return fail(nullptr, st, err);
  return QSP_OK;
}

qsp_status qsp_set_timing(qsp_ctx ctx, int32_t every) {
  return guarded(ctx, [&] {
    if (every < 0) return fail(ctx, QSP_ERR_INVALID_ARG, "every must be >= 0");
    ctx->box->set_timing(every);
    return QSP_OK;
  });
}

qsp_status qsp_get_kernel_times(qsp_ctx ctx, qsp_kernel_times* out) {
  return guarded(ctx, [&] {
    if (!out) return fail(ctx, QSP_ERR_INVALID_ARG, "null output");
    ctx->box->get_kernel_times(out);
    return QSP_OK;
  });
}

qsp_status qsp_get_info(qsp_ctx ctx, int64_t* n_particles, int32_t* cursor) {
  return guarded(ctx, [&] {
    if (n_particles) *n_particles = ctx->box->n_particles();
    if (cursor) *cursor = ctx->box->cursor();
    return QSP_OK;
  });
}

const char* qsp_status_string(qsp_status s) {
  switch (s) {
    case QSP_OK: return "ok";
    case QSP_ERR_INVALID_ARG: return "invalid argument";
    case QSP_ERR_BAD_STATE: return "call out of order";
    case QSP_ERR_OUT_OF_MEMORY: return "out of memory";
    case QSP_ERR_DEVICE: return "device error";
    case QSP_ERR_NONFINITE: return "non-finite value";
  }
  return "unknown status";
}

const char* qsp_last_error(qsp_ctx ctx) {
  return ctx ? ctx->last_error.c_str() : g_last_error.c_str();
}

}  // extern "C"
