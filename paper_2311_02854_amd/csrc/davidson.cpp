// Davidson's method for the lowest eigenpair of the two-dot problem (the
// eigensolver the paper uses in Sec. 2.1).  The subspace vectors V, their
// images W = H V, Gram-Schmidt, residuals and the small projected eigenproblem
// are all FP64 on the GPU; the host keeps only the m x m projected matrix and
// scalars needed for control flow.
//
// Mixed precision: while the residual is large, sigma may run in FP32 or
// split-BF16 (the vectors and everything else stay FP64).  The solver switches
// to FP64 sigma once the residual falls below switch_residual or stops
// improving (its reduced-precision noise floor), restarting from the current
// Ritz vector with an exact image; the energy it returns is always an FP64
// Rayleigh quotient.
#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/dmrg.h"
#include "ops.h"

namespace dmrg {

namespace {
struct DBuf {
  double* p = nullptr;
  explicit DBuf(size_t n) { p = (double*)dev_alloc(std::max<size_t>(1, n) * sizeof(double)); }
  ~DBuf() { dev_free(p); }
};

double ddot(const double* x, const double* y, int64_t n, double* scratch, double* part, void* s) {
  k_multidot(x, 0, 1, y, n, scratch, part, s);
  double v;
  dev_d2h(&v, scratch, sizeof(double), s);
  return v;
}
}  // namespace

int davidson_run(Ops& O, double* psi, const dmrg_davidson_opts& opt, double* energy, dmrg_davidson_stats* st,
                 void* stream, const DavidsonHook& hook) {
  const double t_start = wall_seconds();
  const int64_t n = O.npsi;
  const int mmax = std::max(4, std::min(32, opt.m_max));
  DMRG_CHECK(opt.precision >= 0 && opt.precision <= 2, DMRG_EINVAL, "unknown precision");
  DMRG_CHECK(opt.precond == 0 || (opt.precond == 1 && opt.mlp_weights), DMRG_EINVAL,
             "precond 1 needs mlp_weights");
  DMRG_CHECK(opt.precond_shift >= 0 && std::isfinite(opt.precond_shift), DMRG_EINVAL,
             "precond_shift must be finite and >= 0");
  DBuf V((size_t)mmax * n), W((size_t)mmax * n), dg(n), x(n), hx(n), r(n), t(n), xp(n), hxp(n), sm(4 * 32 * 32 + 64 + (size_t)MULTIDOT_PART * 32);
  double* dvals = sm.p;            // dots
  double* dG = sm.p + 64;          // projected matrix
  double* dw = dG + 32 * 32;       // eigenvalues
  double* dZ = dw + 32;            // eigenvectors
  double* dy = dZ + 32 * 32;       // coefficients
  double* dth = dy + 32;           // theta
  double* dpart = dth + 64;        // partial sums of the dot products (MULTIDOT_PART x 32)
  diag_run(O, dg.p, stream);
  std::vector<double> G(32 * 32, 0.0), y(32, 0.0), yprev(32, 0.0), Z(32 * 32);
  int prec = opt.precision;
  const double floor_ = 1e-8;
  const int stag_max = opt.stagnation > 0 ? opt.stagnation : 4;
  // residual floor of reduced-precision sigma relative to |theta|: a few times
  // the relative sigma error measured for each format
  auto floor_rel = [](int p) { return p == P_F32 ? 6e-6 : (p == P_BF16X3 ? 8e-6 : 0.0); };

  auto sig = [&](const double* in, double* out, int p) { sigma_run(O, in, out, p, stream); };
  auto Vp = [&](int j) { return V.p + (int64_t)j * n; };
  auto Wp = [&](int j) { return W.p + (int64_t)j * n; };

  // v0 = psi / |psi|
  double nrm = std::sqrt(ddot(psi, psi, n, dvals, dpart, stream));
  DMRG_CHECK(nrm > 0 && std::isfinite(nrm), DMRG_EINVAL, "initial vector is zero or not finite");
  k_copy(psi, Vp(0), n, stream);
  k_scale(Vp(0), 1.0 / nrm, n, stream);
  sig(Vp(0), Wp(0), prec);
  int iters = 1, iters64 = (prec == P_F64) ? 1 : 0, switch_iter = (prec == P_F64) ? -1 : 0;
  int m = 1;
  double theta = 0, rn = 1e300, best_rn = 1e300, prev_theta = 1e300, best_any = 1e300;
  int stagnant = 0, ntrace = 0;
  bool have_prev = false, converged = false, reached = false;
  double t_ref = -1;
  int it_ref = -1, fallbacks = 0, mlp_fail = 0;
  bool used_mlp = false;

  auto rebuild_G = [&]() {  // full projected matrix of the current subspace
    for (int j = 0; j < m; ++j) {
      k_multidot(V.p, n, m, Wp(j), n, dvals, dpart, stream);
      std::vector<double> col(m);
      dev_d2h(col.data(), dvals, sizeof(double) * m, stream);
      for (int i = 0; i < m; ++i) G[i * 32 + j] = col[i];
    }
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) G[i * 32 + j] = G[j * 32 + i] = 0.5 * (G[i * 32 + j] + G[j * 32 + i]);
  };
  auto orth_normalize = [&](double* v, int mcur) -> double {
    for (int pass = 0; pass < 2; ++pass) {
      k_multidot(V.p, n, mcur, v, n, dvals, dpart, stream);
      k_sub_lincomb(V.p, n, mcur, dvals, n, v, stream);
    }
    double nv = std::sqrt(ddot(v, v, n, dvals, dpart, stream));
    if (nv > 0 && std::isfinite(nv)) k_scale(v, 1.0 / nv, n, stream);
    return nv;
  };

  rebuild_G();
  for (;;) {
    // projected eigenproblem
    std::vector<double> Gm((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Gm[i * m + j] = G[i * 32 + j];
    dev_h2d_on(dG, Gm.data(), Gm.size() * sizeof(double), stream);
    k_small_eigh(dG, m, m, dw, dZ, stream);
    std::vector<double> wv(m), Zm((size_t)m * m);
    dev_d2h(wv.data(), dw, sizeof(double) * m, stream);
    dev_d2h(Zm.data(), dZ, sizeof(double) * m * m, stream);
    theta = wv[0];
    for (int i = 0; i < m; ++i) y[i] = Zm[i * m + 0];
    dev_h2d_on(dy, y.data(), sizeof(double) * m, stream);
    k_lincomb(V.p, n, m, dy, n, x.p, stream);
    k_lincomb(W.p, n, m, dy, n, hx.p, stream);
    k_copy(hx.p, r.p, n, stream);
    k_axpby(-theta, x.p, 1.0, r.p, n, stream);
    rn = std::sqrt(ddot(r.p, r.p, n, dvals, dpart, stream));
    if (opt.trace && ntrace < opt.trace_cap) {
      double* row = opt.trace + 4 * (int64_t)ntrace++;
      row[0] = wall_seconds() - t_start;
      row[1] = theta;
      row[2] = rn;
      row[3] = prec;
    }
    // the MLP step is judged by the FP64 residual it produced: a step that
    // more than doubles the best residual seen, or is not finite, counts
    // against the model (Davidson residuals are not monotone)
    if (used_mlp && !(rn <= 2.0 * best_any)) ++mlp_fail;
    if (std::isfinite(rn)) best_any = std::min(best_any, rn);
    if (std::isfinite(opt.e_ref) && t_ref < 0 && prec == P_F64 && theta <= opt.e_ref + opt.e_tol) {
      t_ref = wall_seconds() - t_start;
      it_ref = iters;
      reached = true;
    }
    if (prec != P_F64) {
      const bool improving = rn < 0.9 * best_rn || prev_theta - theta > 1e-8 * std::fabs(theta);
      best_rn = std::min(best_rn, rn);
      stagnant = improving ? 0 : stagnant + 1;
    }
    prev_theta = theta;
    const double switch_at = std::max(opt.switch_residual, floor_rel(prec) * std::fabs(theta));
    if (prec != P_F64 && (rn <= switch_at || stagnant >= stag_max)) {
      // switch to FP64 sigma: restart from the Ritz vector and the previous
      // one (as at a subspace restart), both with exact images
      prec = P_F64;
      switch_iter = iters;
      if (have_prev) {
        std::vector<double> yp(m, 0.0);
        for (int i = 0; i < m - 1; ++i) yp[i] = yprev[i];
        dev_h2d_on(dy, yp.data(), sizeof(double) * m, stream);
        k_lincomb(V.p, n, m, dy, n, xp.p, stream);
      }
      k_copy(x.p, Vp(0), n, stream);
      double nx = std::sqrt(ddot(Vp(0), Vp(0), n, dvals, dpart, stream));
      k_scale(Vp(0), 1.0 / nx, n, stream);
      int mnew = 1;
      if (have_prev) {
        k_copy(xp.p, Vp(1), n, stream);
        const double np = orth_normalize(Vp(1), 1);
        if (np > 1e-3 && std::isfinite(np)) mnew = 2;
      }
      for (int j = 0; j < mnew; ++j) {
        sig(Vp(j), Wp(j), prec);
        ++iters;
        ++iters64;
      }
      m = mnew;
      have_prev = false;
      used_mlp = false;
      rn = 1e300;
      best_any = 1e300;
      rebuild_G();
      continue;
    }
    if ((rn <= opt.tol_residual && prec == P_F64) || iters >= opt.max_iter || (reached && opt.stop_at_ref)) {
      converged = rn <= opt.tol_residual && prec == P_F64;
      break;
    }
    // correction vector
    // shifted Ritz value of the preconditioner (the learned one sees it too)
    const double theta_pc = theta - opt.precond_shift * rn;
    dev_h2d_on(dth, &theta_pc, sizeof(double), stream);
    if (hook) hook(x.p, r.p, dg.p, dth, V.p, m, iters);
    used_mlp = opt.precond == 1 && mlp_fail < 3;
    if (used_mlp)
      mlp_precondition(O, r.p, dg.p, dth, t.p, opt.mlp_weights, stream);
    else
      k_precond_diag(r.p, dg.p, dth, floor_, t.p, n, stream);
    if (opt.precond == 1 && !used_mlp) ++fallbacks;
    if (m == mmax) {
      // restart with the current and the previous Ritz vectors
      int mnew = 1;
      if (have_prev) {
        std::vector<double> yp(m, 0.0);
        for (int i = 0; i < m - 1; ++i) yp[i] = yprev[i];
        dev_h2d_on(dy, yp.data(), sizeof(double) * m, stream);
        k_lincomb(V.p, n, m, dy, n, xp.p, stream);
        k_lincomb(W.p, n, m, dy, n, hxp.p, stream);
      }
      k_copy(x.p, Vp(0), n, stream);
      k_copy(hx.p, Wp(0), n, stream);
      if (have_prev) {
        double c = ddot(x.p, xp.p, n, dvals, dpart, stream);
        k_axpby(-c, x.p, 1.0, xp.p, n, stream);
        k_axpby(-c, hx.p, 1.0, hxp.p, n, stream);
        double nx = std::sqrt(ddot(xp.p, xp.p, n, dvals, dpart, stream));
        if (nx > 1e-3) {
          k_copy(xp.p, Vp(1), n, stream);
          k_copy(hxp.p, Wp(1), n, stream);
          k_scale(Vp(1), 1.0 / nx, n, stream);
          k_scale(Wp(1), 1.0 / nx, n, stream);
          mnew = 2;
        }
      }
      m = mnew;
      rebuild_G();
    }
    for (int i = 0; i < 32; ++i) yprev[i] = (i < m) ? y[i] : 0.0;
    have_prev = true;
    k_copy(t.p, Vp(m), n, stream);
    double nt = orth_normalize(Vp(m), m);
    if (!(nt > 1e-14) || !std::isfinite(nt)) {
      // correction collapsed (or the model produced non-finite values): use
      // the residual direction instead
      if (used_mlp) ++mlp_fail;
      k_copy(r.p, Vp(m), n, stream);
      nt = orth_normalize(Vp(m), m);
      if (!(nt > 1e-14)) break;
    }
    sig(Vp(m), Wp(m), prec);
    ++iters;
    if (prec == P_F64) ++iters64;
    ++m;
    // new column/row of the projected matrix
    k_multidot(V.p, n, m, Wp(m - 1), n, dvals, dpart, stream);
    std::vector<double> col(m);
    dev_d2h(col.data(), dvals, sizeof(double) * m, stream);
    for (int i = 0; i < m; ++i) G[i * 32 + (m - 1)] = G[(m - 1) * 32 + i] = col[i];
  }
  k_copy(x.p, psi, n, stream);
  double nx = std::sqrt(ddot(psi, psi, n, dvals, dpart, stream));
  k_scale(psi, 1.0 / nx, n, stream);
  if (prec != P_F64) {
    // stopped before the switch: report the FP64 Rayleigh quotient
    sig(psi, hx.p, P_F64);
    theta = ddot(psi, hx.p, n, dvals, dpart, stream);
    ++iters;
    ++iters64;
  }
  dev_sync(stream);
  *energy = theta;
  if (st) {
    st->iterations = iters;
    st->sigma_fp64 = iters64;
    st->residual = rn;
    st->seconds = wall_seconds() - t_start;
    st->seconds_to_ref = t_ref;
    st->iters_to_ref = it_ref;
    st->mlp_fallbacks = fallbacks;
    st->switch_iter = switch_iter;
    st->trace_len = ntrace;
  }
  return (converged || (reached && opt.stop_at_ref)) ? DMRG_OK : DMRG_ENOCONV;
}

}  // namespace dmrg
