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

double dot(const double* x, const double* y, int64_t n, double* scratch, void* s) {
  k_multidot(x, 0, 1, y, n, scratch, s);
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
  O.mlp_scales = (double*)dev_alloc(sizeof(double) * 2);
  (void)stream;
}

static void mlp_set_weights(Ops& O, const float* w) {
  const int nw = mlp_nweights();
  if (!O.mlp_w) O.mlp_w = (float*)dev_alloc(sizeof(float) * nw);
  if ((int)O.mlp_w_host.size() != nw || std::memcmp(O.mlp_w_host.data(), w, sizeof(float) * nw) != 0) {
    O.mlp_w_host.assign(w, w + nw);
    dev_h2d(O.mlp_w, w, sizeof(float) * nw);
  }
}

void mlp_precondition(Ops& O, const double* r, const double* diag, const double* theta_dev, double* t,
                      const float* weights, void* stream) {
  mlp_prepare(O, stream);
  mlp_set_weights(O, weights);
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
  DBufD x0(n), e(n), d(n), sc(64);
  DBufF ff((size_t)per_iter * NF), fd(per_iter), fy(per_iter);
  int64_t* didx = (int64_t*)dev_alloc(sizeof(int64_t) * std::max(1, per_iter));
  k_copy(psi0, x0.p, n, stream);
  int64_t written = 0;
  std::vector<int64_t> idx(per_iter);
  auto hook = [&](const double* x, const double* r, const double* diag, const double* theta_dev, int iter) {
    if (written >= cap) return;
    // ideal correction: the part of psi_ref orthogonal to x, sign aligned
    const double c = dot(x, psi_ref, n, sc.p, stream);
    k_copy(x, e.p, n, stream);
    k_axpby(c >= 0 ? 1.0 : -1.0, psi_ref, -std::fabs(c), e.p, n, stream);
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
    dev_h2d(didx, idx.data(), sizeof(int64_t) * m);
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

// Adam on the mean squared error of g(f) d - target.
void mlp_train(int64_t n, const float* feat, const float* dcorr, const float* target, int epochs, int batch,
               float lr, uint64_t seed, float* weights, double* loss_before, double* loss_after, void* stream) {
  DMRG_CHECK(n > 0 && epochs >= 0 && batch > 0, DMRG_EINVAL, "training needs n > 0, epochs >= 0, batch > 0");
  const int B = (int)std::min<int64_t>(batch, n);
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

  auto loss_all = [&]() {
    k_mlp_train_fwd(w.p, F.p, n, nullptr, nullptr, g.p, stream);
    k_sqerr(g.p, Dv.p, Y.p, n, sq.p, stream);
    k_sum_f(sq.p, n, one.p, stream);
    float s = 0;
    dev_d2h(&s, one.p, sizeof(float), stream);
    return (double)s / (double)n;
  };
  if (loss_before) *loss_before = loss_all();

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

  std::mt19937_64 rng(seed);
  std::vector<int> perm((size_t)n);
  std::iota(perm.begin(), perm.end(), 0);
  int* dperm = (int*)dev_alloc(sizeof(int) * (size_t)n);
  const float b1 = 0.9f, b2 = 0.999f;
  int64_t step = 0;
  try {
    for (int ep = 0; ep < epochs; ++ep) {
      std::shuffle(perm.begin(), perm.end(), rng);
      dev_h2d(dperm, perm.data(), sizeof(int) * (size_t)n);
      for (int64_t s0 = 0; s0 + B <= n; s0 += B) {
        k_gather_rows(F.p, dperm + s0, B, NF, Fb.p, stream);
        k_gather_rows(Dv.p, dperm + s0, B, 1, Db.p, stream);
        k_gather_rows(Y.p, dperm + s0, B, 1, Yb.p, stream);
        k_mlp_train_fwd(w.p, Fb.p, B, a1.p, a2.p, gb.p, stream);
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
    }
    dev_sync(stream);
  } catch (...) {
    dev_free(dperm);
    throw;
  }
  dev_free(dperm);
  if (loss_after) *loss_after = loss_all();
  dev_d2h(weights, w.p, sizeof(float) * nw, stream);
}

}  // namespace dmrg
