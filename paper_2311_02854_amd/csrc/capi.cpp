// extern "C" entry points of include/dmrg.h.  Every call catches exceptions
// and turns them into status codes plus a per-context message.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>

#include "../../include/dmrg.h"
#include "batch.h"
#include "ops.h"

struct dmrg_ctx {
  int device = 0;
  void* stream = nullptr;
  std::string err;
  std::unique_ptr<dmrg::BatchPlan> batch;  // last fused multi-problem plan
};

struct dmrg_ops {
  std::unique_ptr<dmrg::Ops> p;
};

namespace {
template <typename F>
int guarded(dmrg_ctx* ctx, F&& f) {
  try {
    if (ctx) dmrg::dev_set(ctx->device);
    return f();
  } catch (const dmrg::Error& e) {
    if (ctx) ctx->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return DMRG_EINTERNAL;
  } catch (...) {
    if (ctx) ctx->err = "unknown error";
    return DMRG_EINTERNAL;
  }
}
}  // namespace

extern "C" {

int dmrg_create(dmrg_ctx** ctx, int device, void* hip_stream) {
  if (!ctx) return DMRG_EINVAL;
  *ctx = nullptr;
  auto c = new (std::nothrow) dmrg_ctx();
  if (!c) return DMRG_ENOMEM;
  c->device = device;
  c->stream = hip_stream;
  int rc = guarded(c, [&] {
    dmrg::dev_set(device);
    dmrg::scratch_init(device);  // the static scratch of dmrg_diag_noalloc on this device
    return (int)DMRG_OK;
  });
  if (rc != DMRG_OK) {
    delete c;
    return rc;
  }
  *ctx = c;
  return DMRG_OK;
}

void dmrg_destroy(dmrg_ctx* ctx) { delete ctx; }

const char* dmrg_last_error(const dmrg_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int dmrg_build_ops(dmrg_ctx* ctx, const dmrg_integrals* ints, const dmrg_mps* mps, const dmrg_build_opts* opts,
                   dmrg_ops** out) {
  if (!ctx || !ints || !mps || !out) return DMRG_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&] {
    DMRG_CHECK(ints->K == mps->K && ints->K >= 2, DMRG_EINVAL, "K mismatch between integrals and MPS");
    DMRG_CHECK(ints->h && ints->eri && mps->nsec && mps->sec_qn && mps->sec_dim, DMRG_EINVAL, "null array");
    const int K = ints->K;
    dmrg::Integrals I;
    I.K = K;
    I.h.assign(ints->h, ints->h + (size_t)K * K);
    I.eri.assign(ints->eri, ints->eri + (size_t)K * K * K * K);
    I.ecore = ints->ecore;
    dmrg::BuildOptions opt;
    if (opts && opts->x_budget_bytes) opt.x_budget = opts->x_budget_bytes;
    if (opts && opts->t_budget_bytes) opt.t_budget = opts->t_budget_bytes;
    if (opts && opts->ksplit_tiles) opt.ksplit_tiles = opts->ksplit_tiles;
    DMRG_CHECK(opt.ksplit_tiles > 0, DMRG_EINVAL, "ksplit_tiles must be positive");
    DMRG_CHECK(opt.x_budget >= (size_t(1) << 20) && opt.t_budget >= (size_t(1) << 20), DMRG_EINVAL,
               "scratch budgets below 1 MiB");
    auto o = dmrg::build_ops(I, K, mps->n_alpha, mps->n_beta, mps->bond, mps->nsec, mps->sec_qn, mps->sec_dim,
                             mps->blk_off, mps->data, ctx->stream, opt);
    o->device = ctx->device;
    o->end_call(ctx->stream);
    auto h = new dmrg_ops();
    h->p = std::move(o);
    *out = h;
    return (int)DMRG_OK;
  });
}

void dmrg_ops_destroy(dmrg_ops* ops) {
  if (!ops) return;
  try {
    dmrg::dev_set(ops->p->device);
  } catch (...) {
  }
  delete ops;
}

int dmrg_ops_layout(const dmrg_ops* ops, int64_t* n_psi, int64_t* n_blocks, int* blk_meta, int64_t* blk_off) {
  if (!ops) return DMRG_EINVAL;
  const auto& O = *ops->p;
  if (n_psi) *n_psi = O.npsi;
  if (n_blocks) *n_blocks = (int64_t)O.blocks.size();
  for (size_t i = 0; i < O.blocks.size(); ++i) {
    const auto& b = O.blocks[i];
    if (blk_meta) {
      int* m = blk_meta + 6 * i;
      m[0] = b.il;
      m[1] = b.e / 4;
      m[2] = b.e % 4;
      m[3] = b.ir;
      m[4] = b.dl;
      m[5] = b.dr;
    }
    if (blk_off) blk_off[i] = b.off;
  }
  return DMRG_OK;
}

int dmrg_ops_stats(const dmrg_ops* ops, dmrg_stats* st) {
  if (!ops || !st) return DMRG_EINVAL;
  const auto& O = *ops->p;
  std::memset(st, 0, sizeof(*st));
  st->n_psi = O.npsi;
  st->n_blocks = (int64_t)O.blocks.size();
  st->n_terms = O.nterms;
  st->n_rgemm = O.ngemm_r;
  st->n_lgemm = O.ngemm_l;
  st->flops_rstep = O.flops_r;
  st->flops_lstep = O.flops_l;
  st->flops_sigma = O.flops_r + O.flops_l;
  st->op_bytes = O.op_bytes;
  st->build_seconds = O.build_seconds;
  st->build_flops = O.build_flops;
  st->prof_sigma_calls = O.prof_calls;
  st->prof_launches = O.prof_launches;
  st->prof_gemm_ms = O.prof_ms;
  return DMRG_OK;
}

int dmrg_profile(dmrg_ops* ops, int enable) {
  if (!ops) return DMRG_EINVAL;
  auto& O = *ops->p;
  O.profile = enable != 0;
  O.prof_ms = 0;
  O.prof_launches = O.prof_calls = 0;
  return DMRG_OK;
}

int dmrg_sigma(dmrg_ctx* ctx, dmrg_ops* ops, const double* psi, double* sigma, int precision) {
  if (!ctx || !ops || !psi || !sigma) return DMRG_EINVAL;
  return guarded(ctx, [&] {
    DMRG_CHECK(precision >= 0 && precision <= 2, DMRG_EINVAL, "unknown precision");
    DMRG_CHECK(psi != sigma, DMRG_EINVAL, "psi and sigma must not alias");
    dmrg::Ops& O = *ops->p;
    O.begin_call(ctx->stream);
    dmrg::sigma_run(O, psi, sigma, precision, ctx->stream);
    O.end_call(ctx->stream);
    return (int)DMRG_OK;
  });
}

int dmrg_diag(dmrg_ctx* ctx, dmrg_ops* ops, double* diag) {
  if (!ctx || !ops || !diag) return DMRG_EINVAL;
  return guarded(ctx, [&] {
    dmrg::Ops& O = *ops->p;
    O.begin_call(ctx->stream);
    dmrg::diag_run(O, diag, ctx->stream);
    O.end_call(ctx->stream);
    return (int)DMRG_OK;
  });
}

int dmrg_diag_noalloc(dmrg_ctx* ctx, dmrg_ops* ops, double* diag) {
  if (!ctx || !ops || !diag) return DMRG_EINVAL;
  return guarded(ctx, [&] {
    // calls on one device share its static scratch: one at a time per process
    static std::mutex mu[64];
    DMRG_CHECK(ctx->device >= 0 && ctx->device < 64, DMRG_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(mu[ctx->device]);
    dmrg::Ops& O = *ops->p;
    O.begin_call(ctx->stream);
    dmrg::diag_run_noalloc(O, diag, ctx->stream, dmrg::scratch_get(ctx->device), dmrg::scratch_bytes());
    O.end_call(ctx->stream);
    return (int)DMRG_OK;
  });
}

int dmrg_sigma_batched(dmrg_ctx* ctx, int nprob, dmrg_ops* const* ops, const double* const* psi,
                       double* const* sigma, int precision, int flags) {
  if (!ctx || nprob < 0 || (nprob > 0 && (!ops || !psi || !sigma))) return DMRG_EINVAL;
  if (nprob == 0) return DMRG_OK;
  return guarded(ctx, [&] {
    DMRG_CHECK(precision >= 0 && precision <= 2, DMRG_EINVAL, "unknown precision");
    DMRG_CHECK((flags & ~(DMRG_BATCH_EAGER | DMRG_BATCH_NO_TUNE)) == 0, DMRG_EINVAL, "unknown flags");
    std::vector<dmrg::Ops*> v;
    for (int i = 0; i < nprob; ++i) {
      DMRG_CHECK(ops[i] && psi[i] && sigma[i], DMRG_EINVAL, "null problem entry");
      for (int j = 0; j < i; ++j)
        DMRG_CHECK(ops[j] != ops[i] && sigma[j] != sigma[i], DMRG_EINVAL,
                   "each problem needs its own operators and sigma buffer");
      v.push_back(ops[i]->p.get());
    }
    if (!ctx->batch || !ctx->batch->matches(v, precision)) {
      ctx->batch.reset();
      ctx->batch = dmrg::build_batch(v, precision, ctx->stream);
    }
    for (dmrg::Ops* o : v) o->begin_call(ctx->stream);
    dmrg::BatchPlan& B = *ctx->batch;
    if (!B.tuned && !(flags & DMRG_BATCH_NO_TUNE)) {
      B.bind(psi, sigma, ctx->stream);
      B.autotune(ctx->stream);
    }
    B.run(psi, sigma, !(flags & DMRG_BATCH_EAGER), ctx->stream);
    for (dmrg::Ops* o : v) o->end_call(ctx->stream);
    return (int)DMRG_OK;
  });
}

int dmrg_launch_shape(dmrg_ops* ops, int precision, int tile, int64_t grid_per_xcd) {
  if (!ops || precision < 0 || precision > 2 || tile < 0 || tile >= dmrg::NTILE || grid_per_xcd < -1)
    return DMRG_EINVAL;
  try {
    dmrg::Ops& O = *ops->p;
    O.tile_choice[precision].assign(O.launches.size(), tile);
    O.grid_choice[precision].assign(O.launches.size(), grid_per_xcd);
    return DMRG_OK;
  } catch (...) {
    return DMRG_EINTERNAL;
  }
}

int dmrg_autotune(dmrg_ctx* ctx, dmrg_ops* ops, int precision, double* ms_default, double* ms_tuned) {
  if (!ctx || !ops) return DMRG_EINVAL;
  return guarded(ctx, [&] {
    ops->p->begin_call(ctx->stream);
    dmrg::sigma_autotune(*ops->p, precision, ctx->stream);
    ops->p->end_call(ctx->stream);
    if (ms_default) *ms_default = ops->p->tune_ms_default[precision];
    if (ms_tuned) *ms_tuned = ops->p->tune_ms_best[precision];
    return (int)DMRG_OK;
  });
}

void dmrg_davidson_default_opts(dmrg_davidson_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol_residual = 1e-6;
  o->max_iter = 200;
  o->m_max = 24;
  o->precision = DMRG_FP64;
  o->switch_residual = 1e-4;
  o->stop_at_ref = 0;
  o->stagnation = 4;
  o->trace = nullptr;
  o->trace_cap = 0;
  o->precond = 0;
  o->precond_shift = 1.0;
  o->mlp_weights = nullptr;
  o->e_ref = std::numeric_limits<double>::quiet_NaN();
  o->e_tol = 1e-6;
}

int dmrg_davidson(dmrg_ctx* ctx, dmrg_ops* ops, double* psi, const dmrg_davidson_opts* opts, double* energy,
                  dmrg_davidson_stats* stats) {
  if (!ctx || !ops || !psi || !energy) return DMRG_EINVAL;
  dmrg_davidson_opts o;
  if (opts)
    o = *opts;
  else
    dmrg_davidson_default_opts(&o);
  return guarded(ctx, [&] {
    ops->p->begin_call(ctx->stream);
    int rc = dmrg::davidson_run(*ops->p, psi, o, energy, stats, ctx->stream);
    ops->p->end_call(ctx->stream);
    return rc;
  });
}

int dmrg_decimate(dmrg_ctx* ctx, dmrg_ops* ops, const double* psi, int D, int direction, double cutoff,
                  dmrg_decimation_info* out) {
  if (!ctx || !ops || !psi || !out) return DMRG_EINVAL;
  return guarded(ctx, [&] {
    dmrg::Ops& O = *ops->p;
    O.begin_call(ctx->stream);
    dmrg::decimate_run(O, psi, D, direction, cutoff, ctx->stream);
    O.end_call(ctx->stream);
    const dmrg::Decimation& R = *O.decim;
    out->nsec = (int)R.sec.size();
    out->nblk = (int64_t)R.blk_off.size();
    out->ndata = (int64_t)R.data.size();
    out->kept = 0;
    for (int d : R.dim) out->kept += d;
    out->discarded = R.discarded;
    out->entropy = R.entropy;
    return (int)DMRG_OK;
  });
}

int dmrg_decimation_get(const dmrg_ops* ops, int* sec_qn, int* sec_dim, int64_t* blk_off, double* data) {
  if (!ops || !ops->p->decim) return DMRG_EINVAL;
  const dmrg::Decimation& R = *ops->p->decim;
  for (size_t i = 0; i < R.sec.size(); ++i) {
    if (sec_qn) {
      sec_qn[2 * i] = R.sec[i].a;
      sec_qn[2 * i + 1] = R.sec[i].b;
    }
    if (sec_dim) sec_dim[i] = R.dim[i];
  }
  if (blk_off) std::copy(R.blk_off.begin(), R.blk_off.end(), blk_off);
  if (data) std::copy(R.data.begin(), R.data.end(), data);
  return DMRG_OK;
}

int dmrg_mlp_nweights(void) { return dmrg::mlp_nweights(); }

int dmrg_mlp_init(float* weights, uint64_t seed) {
  if (!weights) return DMRG_EINVAL;
  dmrg::mlp_init(weights, seed);
  return DMRG_OK;
}

int dmrg_mlp_collect(dmrg_ctx* ctx, dmrg_ops* ops, const double* psi0, const double* psi_ref, int max_iter,
                     int per_iter, uint64_t seed, int64_t cap, float* feat, float* dcorr, float* target,
                     int64_t* n_out) {
  if (!ctx || !ops || !psi0 || !psi_ref || !feat || !dcorr || !target || !n_out) return DMRG_EINVAL;
  return guarded(ctx, [&] {
    DMRG_CHECK(max_iter > 0 && per_iter > 0 && cap >= 0, DMRG_EINVAL, "max_iter, per_iter > 0 and cap >= 0 needed");
    ops->p->begin_call(ctx->stream);
    *n_out = dmrg::mlp_collect(*ops->p, psi0, psi_ref, max_iter, per_iter, seed, cap, feat, dcorr, target,
                               ctx->stream);
    ops->p->end_call(ctx->stream);
    return (int)DMRG_OK;
  });
}

int dmrg_mlp_train(dmrg_ctx* ctx, int64_t n, const float* feat, const float* dcorr, const float* target, int group,
                   int epochs, int batch, float lr, uint64_t seed, float* weights, double* loss_before,
                   double* loss_after) {
  if (!ctx || !feat || !dcorr || !target || !weights) return DMRG_EINVAL;
  return guarded(ctx, [&] {
    dmrg::mlp_train(n, feat, dcorr, target, group, epochs, batch, lr, seed, weights, loss_before, loss_after,
                    ctx->stream);
    return (int)DMRG_OK;
  });
}

int dmrg_mlp_apply(dmrg_ctx* ctx, dmrg_ops* ops, const float* weights, const double* r, const double* diag,
                   double theta, double* t) {
  if (!ctx || !ops || !weights || !r || !diag || !t) return DMRG_EINVAL;
  return guarded(ctx, [&] {
    ops->p->begin_call(ctx->stream);
    dmrg::mlp_apply_once(*ops->p, weights, r, diag, theta, t, ctx->stream);
    ops->p->end_call(ctx->stream);
    return (int)DMRG_OK;
  });
}

}  // extern "C"

