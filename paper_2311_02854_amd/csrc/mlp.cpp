// Learned Davidson preconditioner (an addition to the paper's method, whose
// Davidson solver, Sec. 2.1, uses no preconditioner model): per-element gains
// g = MLP(features) on the diagonal correction r_i / (theta - H_ii), trained
// on pairs (features, diagonal correction, ideal correction) that Davidson
// runs on the method's own problems generate.  Layout of features and
// weights: include/dmrg.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "ops.h"

namespace dmrg {

namespace {
constexpr int NF = DMRG_MLP_NFEAT, HD = DMRG_MLP_HIDDEN, NS = NF - 4;
constexpr double FLOOR = 1e-8;

struct DBufD {
  double* p = nullptr;
  explicit DBufD(size_t n) { p = (double*)dev_alloc(std::max<size_t>(1, n) * sizeof(double)); }
  ~DBufD() { dev_free(p); }
};
struct DBufF {
  float* p = nullptr;
  explicit DBufF(size_t n) { p = (float*)dev_alloc(std::max<size_t>(1, n) * sizeof(float)); }
  ~DBufF() { dev_free(p); }
};

// scratch: 1 + MULTIDOT_PART doubles (result, then the partial sums)
double dot(const double* x, const double* y, int64_t n, double* scratch, void* s) {
  k_multidot(x, 0, 1, y, n, scratch, scratch + 1, s);
  double v;
  dev_d2h(&v, scratch, sizeof(double), s);
  return v;
}
}  // namespace

int mlp_nweights() { return NF * HD + HD + HD * HD + HD + HD + 1; }

void mlp_init(float* w, uint64_t seed) {
  std::mt19937_64 rng(seed);
  auto uni = [&](double a) { return (float)(std::uniform_real_distribution<double>(-a, a)(rng)); };
  float* p = w;
  const double a1 = std::sqrt(6.0 / NF), a2 = std::sqrt(6.0 / HD);
  for (int i = 0; i < NF * HD; ++i) *p++ = uni(a1);
  for (int i = 0; i < HD; ++i) *p++ = 0.f;
  for (int i = 0; i < HD * HD; ++i) *p++ = uni(a2);
  for (int i = 0; i < HD; ++i) *p++ = 0.f;
  for (int i = 0; i < HD; ++i) *p++ = 0.f;  // w3
  *p++ = 1.f;                                // b3: g = 1
}

// Per-element block index and per-block static features (columns 4..17).
void mlp_prepare(Ops& O, void* stream) {
  if (O.mlp_blk) return;
  const int nb = (int)O.blocks.size();
  std::vector<int> blk((size_t)O.npsi);
  std::vector<float> stat((size_t)nb * NS, 0.f);
  const double K = O.K, k = O.bond, rK = std::sqrt(K);
  for (int b = 0; b < nb; ++b) {
    const PsiBlk& B = O.blocks[b];
    std::fill(blk.begin() + B.off, blk.begin() + B.off + (int64_t)B.dl * B.dr, b);
    float* s = &stat[(size_t)b * NS];
    const QN ql = O.Llabel[B.il], qr = O.Rlabel[B.ir];
    s[0] = (float)((ql.a - O.Na * k / K) / rK);
    s[1] = (float)((ql.b - O.Nb * k / K) / rK);
    s[2] = (float)(((O.Na - qr.a) - O.Na * (K - k - 2) / K) / rK);
    s[3] = (float)(((O.Nb - qr.b) - O.Nb * (K - k - 2) / K) / rK);
    s[4 + B.e / 4] = 1.f;
    s[8 + B.e % 4] = 1.f;
    s[12] = (float)(std::log2((double)B.dl) / 10.0);
    s[13] = (float)(std::log2((double)B.dr) / 10.0);
  }
  O.mlp_blk = (int*)dev_alloc(sizeof(int) * blk.size());
  dev_h2d(O.mlp_blk, blk.data(), sizeof(int) * blk.size());
  O.mlp_stat = (float*)dev_alloc(sizeof(float) * stat.size());
  dev_h2d(O.mlp_stat, stat.data(), sizeof(float) * stat.size());
  O.mlp_part = (double*)dev_alloc(sizeof(double) * 2 * 256);
  O.mlp_scales = (double*)dev_alloc(sizeof(double) * 4);
  (void)stream;
}

static void mlp_set_weights(Ops& O, const float* w, void* stream) {
  const int nw = mlp_nweights();
  if (!O.mlp_w) O.mlp_w = (float*)dev_alloc(sizeof(float) * nw);
  if ((int)O.mlp_w_host.size() != nw || std::memcmp(O.mlp_w_host.data(), w, sizeof(float) * nw) != 0) {
    O.mlp_w_host.assign(w, w + nw);
    dev_h2d_on(O.mlp_w, w, sizeof(float) * nw, stream);  // after the applies already queued
  }
}

void mlp_precondition(Ops& O, const double* r, const double* diag, const double* theta_dev, double* t,
                      const float* weights, void* stream) {
  mlp_prepare(O, stream);
  mlp_set_weights(O, weights, stream);
  k_mlp_scales(r, diag, theta_dev, O.npsi, O.mlp_part, O.mlp_scales, stream);
  k_mlp_apply(O.mlp_w, r, diag, theta_dev, O.mlp_scales, O.mlp_blk, O.mlp_stat, FLOOR, t, O.npsi, stream);
}

void mlp_apply_once(Ops& O, const float* weights, const double* r, const double* diag, double theta, double* t,
                    void* stream) {
  DBufD th(1);
  dev_h2d(th.p, &theta, sizeof(double));
  mlp_precondition(O, r, diag, th.p, t, weights, stream);
  dev_sync(stream);
}

int64_t mlp_collect(Ops& O, const double* psi0, const double* psi_ref, int max_iter, int per_iter, uint64_t seed,
                    int64_t cap, float* feat, float* dcorr, float* target, void* stream) {
  mlp_prepare(O, stream);
  const int64_t n = O.npsi;
  DBufD x0(n), e(n), d(n), sc(1 + MULTIDOT_PART), dots(64), part((size_t)MULTIDOT_PART * 64);
  DBufF ff((size_t)per_iter * NF), fd(per_iter), fy(per_iter);
  int64_t* didx = (int64_t*)dev_alloc(sizeof(int64_t) * std::max(1, per_iter));
  k_copy(psi0, x0.p, n, stream);
  int64_t written = 0;
  std::vector<int64_t> idx(per_iter);
  auto hook = [&](const double* x, const double* r, const double* diag, const double* theta_dev, const double* V,
                  int m_sub, int iter) {
    if (written >= cap) return;
    (void)x;
    // ideal correction: the part of psi_ref orthogonal to the current subspace
    // (which holds the Ritz vector), i.e. what the next direction must supply;
    // two projection passes
    k_copy(psi_ref, e.p, n, stream);
    for (int pass = 0; pass < 2; ++pass) {
      k_multidot(V, n, m_sub, e.p, n, dots.p, part.p, stream);
      k_sub_lincomb(V, n, m_sub, dots.p, n, e.p, stream);
    }
    k_precond_diag(r, diag, theta_dev, FLOOR, d.p, n, stream);
    const double de = dot(d.p, e.p, n, sc.p, stream), ee = dot(e.p, e.p, n, sc.p, stream);
    const double dd = dot(d.p, d.p, n, sc.p, stream);
    if (!(ee > 0) || !(dd > 0)) return;
    const double rms_d = std::sqrt(dd / (double)n);
    // d and target are both divided by rms(d) so that every iteration weighs alike
    const double es = de / ee / rms_d;
    k_mlp_scales(r, diag, theta_dev, n, O.mlp_part, O.mlp_scales, stream);
    std::mt19937_64 rng(seed * 1000003ULL + (uint64_t)iter);
    std::uniform_int_distribution<int64_t> U(0, n - 1);
    const int m = (int)std::min<int64_t>(per_iter, cap - written);
    for (int j = 0; j < m; ++j) idx[j] = U(rng);
    dev_h2d_on(didx, idx.data(), sizeof(int64_t) * m, stream);
    k_mlp_gather_pairs(didx, m, r, diag, theta_dev, O.mlp_scales, O.mlp_blk, O.mlp_stat, e.p, es, FLOOR, ff.p,
                       fd.p, fy.p, stream);
    // k_mlp_gather_pairs computes d_i from r; rescale it by rms(d) like the target
    std::vector<float> hf((size_t)m * NF), hd(m), hy(m);
    dev_d2h(hf.data(), ff.p, sizeof(float) * hf.size(), stream);
    dev_d2h(hd.data(), fd.p, sizeof(float) * m, stream);
    dev_d2h(hy.data(), fy.p, sizeof(float) * m, stream);
    for (int j = 0; j < m; ++j) hd[j] = (float)(hd[j] / rms_d);
    std::memcpy(feat + written * NF, hf.data(), sizeof(float) * hf.size());
    std::memcpy(dcorr + written, hd.data(), sizeof(float) * m);
    std::memcpy(target + written, hy.data(), sizeof(float) * m);
    written += m;
  };
  dmrg_davidson_opts o;
  dmrg_davidson_default_opts(&o);
  o.tol_residual = 1e-9;
  o.max_iter = max_iter;
  o.precision = DMRG_FP64;
  o.precond = 0;
  double en = 0;
  try {
    davidson_run(O, x0.p, o, &en, nullptr, stream, hook);
  } catch (...) {
    dev_free(didx);
    throw;
  }
  dev_free(didx);
  return written;
}

// Training by Adam.  Loss, for group == 0: mean_i (g(f_i) d_i - target_i)^2
// over minibatches of `batch` pairs; for group > 0: the pairs form groups of
// `group` consecutive entries (the samples of one Davidson iteration) and the
// loss of a group is the direction loss 1 - cos^2(g.d, target), which does not
// depend on the scale of the correction; one group per step.  A seeded tenth
// of the pairs (of the groups) is held out; after every epoch the held-out loss
// decides whether the weights are kept, starting from the given ones, so the
// result is never worse on held-out data than the start (g = 1 for the
// dmrg_mlp_init weights).
void mlp_train(int64_t n, const float* feat, const float* dcorr, const float* target, int group, int epochs,
               int batch, float lr, uint64_t seed, float* weights, double* loss_before, double* loss_after,
               void* stream) {
  DMRG_CHECK(n > 1 && epochs >= 0 && group >= 0 && (group > 0 || batch > 0), DMRG_EINVAL,
             "training needs n > 1, epochs >= 0, and a batch or group size");
  DMRG_CHECK(group == 0 || (n % group == 0 && n / group >= 2 && group <= (1 << 16)), DMRG_EINVAL,
             "n must be a multiple of group, with at least two groups");
  const bool cosl = group > 0;
  // units: single pairs (MSE) or groups (direction loss)
  const int64_t usz = cosl ? group : 1, nunit = n / usz;
  const int64_t nval = std::max<int64_t>(1, nunit / 10), ntr = nunit - nval;
  const int B = cosl ? group : (int)std::min<int64_t>(batch, ntr);
  const int nw = mlp_nweights();
  DBufF F((size_t)n * NF), Dv(n), Y(n), g(n), sq(n);
  DBufF Fb((size_t)B * NF), Db(B), Yb(B), a1((size_t)B * HD), a2((size_t)B * HD), gb(B), dout(B),
      dz2((size_t)B * HD), da1((size_t)B * HD), grad(nw), m(nw), v(nw), w(nw), one(1);
  dev_h2d(F.p, feat, sizeof(float) * (size_t)n * NF);
  dev_h2d(Dv.p, dcorr, sizeof(float) * n);
  dev_h2d(Y.p, target, sizeof(float) * n);
  dev_h2d(w.p, weights, sizeof(float) * nw);
  float* gW1 = grad.p;
  float* gb1 = gW1 + NF * HD;
  float* gW2 = gb1 + HD;
  float* gb2 = gW2 + HD * HD;
  float* gw3 = gb2 + HD;
  float* gb3 = gw3 + HD;
  const float* W2 = w.p + NF * HD + HD;

  std::mt19937_64 rng(seed);
  std::vector<int> uperm((size_t)nunit);
  std::iota(uperm.begin(), uperm.end(), 0);
  std::shuffle(uperm.begin(), uperm.end(), rng);
  std::vector<char> is_val((size_t)nunit, 0);
  for (int64_t u = ntr; u < nunit; ++u) is_val[uperm[u]] = 1;

  // loss over the held-out units (val) or all units, from one forward pass
  std::vector<float> hg((size_t)n);
  auto eval = [&](bool val_only) {
    k_mlp_train_fwd(w.p, F.p, n, nullptr, nullptr, g.p, stream);
    dev_d2h(hg.data(), g.p, sizeof(float) * (size_t)n, stream);
    double tot = 0;
    int64_t cnt = 0;
    for (int64_t u = 0; u < nunit; ++u) {
      if (val_only && !is_val[u]) continue;
      double A = 0, T = 0, Yy = 0, se = 0;
      for (int64_t i = u * usz; i < (u + 1) * usz; ++i) {
        const double t = (double)hg[i] * dcorr[i];
        A += t * target[i];
        T += t * t;
        Yy += (double)target[i] * target[i];
        se += (t - target[i]) * (t - target[i]);
      }
      tot += cosl ? 1.0 - A * A / ((T + 1e-300) * (Yy + 1e-300)) : se;
      cnt += cosl ? 1 : usz;
    }
    return tot / (double)std::max<int64_t>(1, cnt);
  };
  if (loss_before) *loss_before = eval(false);
  std::vector<float> best(weights, weights + nw);
  double best_val = eval(true);

  // the three training GEMMs on the grouped FP32 kernel (ids >= 2 only)
  DevTable tab;
  const int i_a1 = tab.add(a1.p), i_dz2 = tab.add(dz2.p), i_da1 = tab.add(da1.p), i_Fb = tab.add(Fb.p);
  const int i_gW2 = tab.add(gW2), i_gW1 = tab.add(gW1), i_W2 = tab.add(const_cast<float*>(W2));
  GemmList gW2l, da1l, gW1l;
  gW2l.begin(HD, HD, 1, i_gW2, 0, HD, 0, false);   // dW2 = a1^T dz2
  gW2l.add(make_contrib(B, GF_TRANS_A, i_a1, 0, HD, i_dz2, 0, HD, 1.0));
  gW2l.end();
  da1l.begin(B, HD, 1, i_da1, 0, HD, 0, false);    // da1 = dz2 W2^T
  da1l.add(make_contrib(HD, GF_TRANS_B, i_dz2, 0, HD, i_W2, 0, HD, 1.0));
  da1l.end();
  gW1l.begin(NF, HD, 1, i_gW1, 0, HD, 0, false);   // dW1 = Fb^T dz1
  gW1l.add(make_contrib(B, GF_TRANS_A, i_Fb, 0, NF, i_da1, 0, HD, 1.0));
  gW1l.end();

  // rows of each step: a contiguous group, or a shuffled minibatch of pairs
  std::vector<int> rows((size_t)n);
  int* drows = (int*)dev_alloc(sizeof(int) * (size_t)n);
  const float b1 = 0.9f, b2 = 0.999f;
  int64_t step = 0;
  try {
    for (int ep = 0; ep < epochs; ++ep) {
      std::vector<int> tr;
      for (int64_t u = 0; u < nunit; ++u)
        if (!is_val[u]) tr.push_back((int)u);
      std::shuffle(tr.begin(), tr.end(), rng);
      int64_t nr = 0;
      for (int u : tr)
        for (int64_t i = 0; i < usz; ++i) rows[nr++] = (int)(u * usz + i);
      dev_h2d_on(drows, rows.data(), sizeof(int) * (size_t)nr, stream);
      for (int64_t s0 = 0; s0 + B <= nr; s0 += B) {
        k_gather_rows(F.p, drows + s0, B, NF, Fb.p, stream);
        k_gather_rows(Dv.p, drows + s0, B, 1, Db.p, stream);
        k_gather_rows(Y.p, drows + s0, B, 1, Yb.p, stream);
        k_mlp_train_fwd(w.p, Fb.p, B, a1.p, a2.p, gb.p, stream);
        if (cosl)
          k_mlp_cos_grad(w.p, gb.p, Db.p, Yb.p, a2.p, B, dout.p, dz2.p, sq.p, stream);
        else
          k_mlp_bwd_out(w.p, gb.p, Db.p, Yb.p, a2.p, B, dout.p, dz2.p, stream);
        k_colsum(a2.p, dout.p, B, HD, gw3, stream);
        k_sum_f(dout.p, B, gb3, stream);
        k_colsum(dz2.p, nullptr, B, HD, gb2, stream);
        gW2l.run(tab, nullptr, nullptr, P_F32, stream);
        da1l.run(tab, nullptr, nullptr, P_F32, stream);
        k_relu_mask(da1.p, a1.p, (int64_t)B * HD, stream);
        gW1l.run(tab, nullptr, nullptr, P_F32, stream);
        k_colsum(da1.p, nullptr, B, HD, gb1, stream);
        ++step;
        const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
        k_adam(w.p, grad.p, m.p, v.p, nw, lr, b1, b2, c1, c2, 1e-8f, stream);
      }
      const double val = eval(true);
      if (val < best_val) {
        best_val = val;
        dev_d2h(best.data(), w.p, sizeof(float) * nw, stream);
      }
    }
    dev_sync(stream);
  } catch (...) {
    dev_free(drows);
    throw;
  }
  dev_free(drows);
  std::copy(best.begin(), best.end(), weights);
  dev_h2d(w.p, weights, sizeof(float) * nw);
  if (loss_after) *loss_after = eval(false);
}

}  // namespace dmrg
