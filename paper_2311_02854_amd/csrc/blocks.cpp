// Growth of a renormalized block by one site (Eq. Renorm), on the GPU.
//
// A block carries the normal operators of its own spin orbitals (a+_p, A_pq,
// B_ps), S_p for every external p and H (the qops set of Eq. qops restricted
// to normal operators; complementary P and Q are formed from A and B as
// exact linear combinations wherever they are needed).  The operators of the
// enlarged block Z = X (x) site (left growth) or site (x) X (right growth)
// are sums of products O1.O2 (O1 on the first factor in Jordan-Wigner order);
// each product acts on |z1 z2> with the sign (-1)^(parity(O2) N(z1)).  A term
// family applies one such product, with a fixed site matrix, to a run of
// group members; its projection with the site tensor is two batched GEMM
// phases:
//   left:  T = X(l',l) A(l,n,r),   O_new(r',r) += c s(n',n) zeta(l) A(l',n',r')^T T
//   right: T = X(r',r) A(l,n,r)^T, O_new(l',l) += c s(n',n) zeta(n) A(l',n',r') T
#include "blocks.h"

#include <algorithm>
#include <cmath>

namespace dmrg {

static const QN GROUP_DQ[NG] = {QN(1, 0),  QN(0, 1),  QN(2, 0),  QN(1, 1),  QN(0, 2), QN(0, 0),
                                QN(1, -1), QN(-1, 1), QN(-1, 0), QN(0, -1), QN(0, 0)};
static const int GROUP_PAR[NG] = {1, 1, 0, 0, 0, 0, 0, 0, 1, 1, 0};

std::string key_str(const OpKey& k) {
  return std::string(1, k.kind) + "(" + std::to_string(k.p) + "," + std::to_string(k.q) + ")";
}

// ------------------------------------------------------------------ site ops
namespace site {
Mat4 I() {
  Mat4 m{};
  for (int i = 0; i < 4; ++i) m[i * 4 + i] = 1.0;
  return m;
}
Mat4 cre(int spin) {
  Mat4 m{};
  if (spin == 0) {      // a+_alpha: |vac> -> |alpha>, |beta> -> a+_a a+_b |vac> = |alpha beta>
    m[2 * 4 + 0] = 1.0;
    m[3 * 4 + 1] = 1.0;
  } else {              // a+_beta: |vac> -> |beta>, |alpha> -> a+_b a+_a |vac> = -|alpha beta>
    m[1 * 4 + 0] = 1.0;
    m[3 * 4 + 2] = -1.0;
  }
  return m;
}
Mat4 tr(const Mat4& a) {
  Mat4 m{};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m[i * 4 + j] = a[j * 4 + i];
  return m;
}
Mat4 ann(int spin) { return tr(cre(spin)); }
Mat4 mul(const Mat4& a, const Mat4& b) {
  Mat4 m{};
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 4; ++j) m[i * 4 + j] += a[i * 4 + k] * b[k * 4 + j];
  return m;
}
Mat4 scale(const Mat4& a, double s) {
  Mat4 m = a;
  for (auto& x : m) x *= s;
  return m;
}
bool zero(const Mat4& a) {
  for (double x : a)
    if (x != 0.0) return false;
  return true;
}
int nelec(int n) { return SITE_QN[n].n(); }
}  // namespace site

// ------------------------------------------------------------------ groups
void Group::alloc(DevTable& tab, void* stream, DeviceArena* arena) {
  size_t cnt = (size_t)std::max<int64_t>(1, (int64_t)n() * lay.size);
  dev = (double*)(arena ? arena->take(cnt * sizeof(double)) : dev_alloc_nozero(cnt * sizeof(double)));
  in_arena = arena != nullptr;
  k_zero_bytes(dev, cnt * sizeof(double), stream);
  buf = tab.add(dev);
}
void Group::free_dev() {
  if (!in_arena) dev_free(dev);
  dev = nullptr;
  dev_free(dev32);
  dev32 = nullptr;
}

int Block::member(int gid, OpKey k) const {
  const auto& nm = g[gid].names;
  for (int i = 0; i < (int)nm.size(); ++i)
    if (nm[i].kind == k.kind && nm[i].p == k.p && nm[i].q == k.q) return i;
  return -1;
}

void Builder::run(GemmList& gl) {
  if (gl.empty()) return;
  gl.upload(gl.tile, nullptr, ring.get());
  gl.run_uploaded(gl.tile, tab.device(*ring), nullptr, nullptr, P_F64, stream);
  st.flops += gl.flops;
  st.ngemm += gl.ngemm;
}

std::unique_ptr<Block> Builder::vacuum(bool left) {
  auto B = std::make_unique<Block>();
  B->left = left;
  B->nsites = 0;
  B->first_site = left ? 0 : I.K;
  B->basis.qn = {QN(0, 0)};
  B->basis.dim = {1};
  B->basis.finish();
  B->g.resize(NG);
  for (int gid = 0; gid < NG; ++gid) {
    B->g[gid].dq = GROUP_DQ[gid];
    B->g[gid].parity = GROUP_PAR[gid];
    B->g[gid].lay = make_layout(B->basis, GROUP_DQ[gid]);
  }
  for (int i = 0; i < I.K; ++i) {
    B->ext_a.push_back(2 * i);
    B->ext_b.push_back(2 * i + 1);
    B->g[G_SA].names.push_back({'S', 2 * i, -1});
    B->g[G_SB].names.push_back({'S', 2 * i + 1, -1});
  }
  B->g[G_H].names.push_back({'H', -1, -1});
  for (auto& x : B->g) x.alloc(tab, stream);  // zero-filled: S = 0, H = 0 on the empty block
  return B;
}

std::unique_ptr<Group> Builder::combine(const Group& src, const std::vector<std::vector<double>>& coef,
                                        std::vector<OpKey> names, bool scratch) {
  auto G = std::make_unique<Group>();
  G->dq = src.dq;
  G->parity = src.parity;
  G->lay = src.lay;
  G->names = std::move(names);
  G->alloc(tab, stream, scratch ? &step_arena : nullptr);
  const int nout = (int)coef.size(), nin = src.n();
  if (nout == 0 || nin == 0 || src.lay.size == 0) return G;
  std::vector<double> c((size_t)nout * nin);
  for (int r = 0; r < nout; ++r)
    for (int m = 0; m < nin; ++m) c[(size_t)r * nin + m] = coef[r][m];
  // the coefficients are read by the launch below only: staged in the ring
  double* dc = (double*)ring->put(c.data(), c.size() * sizeof(double));
  int cb = tab.add(dc);
  GemmList gl;
  // out (nout x S) = C (nout x nin) * src (nin x S); split N so a task stays < 2^31 elements
  const int64_t S = src.lay.size;
  const int64_t NCH = int64_t(1) << 20;
  for (int64_t n0 = 0; n0 < S; n0 += NCH) {
    int nn = (int)std::min<int64_t>(NCH, S - n0);
    gl.begin(nout, nn, 1, G->buf, n0, (int)S, 0, false);
    gl.add(make_contrib(nin, 0, cb, 0, nin, src.buf, n0, (int)S, 1.0));
    gl.end();
  }
  run(gl);
  tab.set(cb, nullptr);
  return G;
}

// ------------------------------------------------------------------ growth
namespace {

struct Fam {
  int out = 0, out_base = 0, count = 0;
  const Group* src = nullptr;  // nullptr: identity on the block
  int src_base = 0;
  bool trans = false;
  Mat4 s{};
  int pi = 0;                  // parity of the second factor (JW sign)
  double coef = 1.0;
  std::vector<double> cv;      // optional per-member coefficients
};

// effective block of op(src) with ket sector `ket`: returns stored block index or -1
inline int eff_block(const Layout& lay, bool trans, int ket, int* bra) {
  if (!trans) {
    int k = lay.by_ket[ket];
    if (k >= 0) *bra = lay.bra[k];
    return k;
  }
  int k = lay.by_bra[ket];
  if (k >= 0) *bra = lay.ket[k];
  return k;
}

int spin(int p) { return p & 1; }

}  // namespace

std::unique_ptr<Block> Builder::grow(const Block& X, int j, const SiteTensor& A, const Basis& newbasis,
                                     bool last) {
  const bool left = X.left;
  const int aj = 2 * j, bj = 2 * j + 1;
  auto Zp = std::make_unique<Block>();
  Block& Z = *Zp;
  Z.left = left;
  Z.nsites = X.nsites + 1;
  Z.first_site = left ? 0 : j;
  Z.basis = newbasis;
  Z.g.resize(NG);
  const auto& xa = X.g[G_CA].names;
  const auto& xb = X.g[G_CB].names;
  const int nXa = (int)xa.size(), nXb = (int)xb.size();

  // ---- member lists of Z (inherited first for left growth, new first for right)
  auto cat = [&](int gid, std::vector<OpKey> fresh) {
    auto& out = Z.g[gid].names;
    const auto& old = X.g[gid].names;
    if (left) {
      out = old;
      out.insert(out.end(), fresh.begin(), fresh.end());
    } else {
      out = fresh;
      out.insert(out.end(), old.begin(), old.end());
    }
  };
  auto keys = [](char kind, const std::vector<OpKey>& ps, int other, bool other_second) {
    std::vector<OpKey> v;
    for (auto& k : ps) v.push_back(other_second ? OpKey{kind, k.p, other} : OpKey{kind, other, k.p});
    return v;
  };
  auto join = [](std::initializer_list<std::vector<OpKey>> parts) {
    std::vector<OpKey> v;
    for (auto& p : parts) v.insert(v.end(), p.begin(), p.end());
    return v;
  };
  cat(G_CA, {{'C', aj, -1}});
  cat(G_CB, {{'C', bj, -1}});
  if (left) {
    cat(G_AAA, keys('A', xa, aj, true));
    cat(G_ABB, keys('A', xb, bj, true));
    cat(G_AAB, join({keys('A', xa, bj, true), keys('A', xb, aj, true), {{'A', aj, bj}}}));
    cat(G_B0, join({keys('B', xa, aj, true), keys('B', xa, aj, false), {{'B', aj, aj}},
                    keys('B', xb, bj, true), keys('B', xb, bj, false), {{'B', bj, bj}}}));
    cat(G_BAB, join({keys('B', xa, bj, true), keys('B', xb, aj, false), {{'B', aj, bj}}}));
    cat(G_BBA, join({keys('B', xb, aj, true), keys('B', xa, bj, false), {{'B', bj, aj}}}));
  } else {
    cat(G_AAA, keys('A', xa, aj, false));
    cat(G_ABB, keys('A', xb, bj, false));
    cat(G_AAB, join({keys('A', xb, aj, false), keys('A', xa, bj, false), {{'A', aj, bj}}}));
    cat(G_B0, join({keys('B', xa, aj, false), keys('B', xa, aj, true), {{'B', aj, aj}},
                    keys('B', xb, bj, false), keys('B', xb, bj, true), {{'B', bj, bj}}}));
    cat(G_BAB, join({keys('B', xb, aj, false), keys('B', xa, bj, true), {{'B', aj, bj}}}));
    cat(G_BBA, join({keys('B', xa, bj, false), keys('B', xb, aj, true), {{'B', bj, aj}}}));
  }
  // S: the site's modes leave the external set (first externals for left
  // growth, last ones for right growth)
  auto drop = [&](const std::vector<int>& ext, int mode) {
    std::vector<int> v;
    for (int m : ext)
      if (m != mode) v.push_back(m);
    return v;
  };
  Z.ext_a = drop(X.ext_a, aj);
  Z.ext_b = drop(X.ext_b, bj);
  const int sa_base = left ? 1 : 0, sb_base = left ? 1 : 0;
  DMRG_CHECK(X.ext_a.size() == Z.ext_a.size() + 1 && X.ext_b.size() == Z.ext_b.size() + 1, DMRG_EINTERNAL,
             "external mode bookkeeping");
  DMRG_CHECK(left ? (X.ext_a[0] == aj && X.ext_b[0] == bj) : (X.ext_a.back() == aj && X.ext_b.back() == bj),
             DMRG_EINTERNAL, "site is not adjacent to the block");
  for (int m : Z.ext_a) Z.g[G_SA].names.push_back({'S', m, -1});
  for (int m : Z.ext_b) Z.g[G_SB].names.push_back({'S', m, -1});
  Z.g[G_H].names.push_back({'H', -1, -1});
  size_t zbytes = 0;
  for (int gid = 0; gid < NG; ++gid) {
    Z.g[gid].dq = GROUP_DQ[gid];
    Z.g[gid].parity = GROUP_PAR[gid];
    Z.g[gid].lay = make_layout(Z.basis, GROUP_DQ[gid]);
    zbytes += ((size_t)std::max<int64_t>(1, (int64_t)Z.g[gid].n() * Z.g[gid].lay.size) * sizeof(double) + 255) &
              ~size_t(255);
  }
  if (!last) {
    Z.arena.reset(new DeviceArena());
    Z.arena->reserve(zbytes);
  }
  for (int gid = 0; gid < NG; ++gid) Z.g[gid].alloc(tab, stream, Z.arena.get());

  // ---- families
  using namespace site;
  const Mat4 I4 = site::I(), CA = cre(0), CB = cre(1), AA = ann(0), AB = ann(1);
  const Mat4 CRE[2] = {CA, CB}, ANN[2] = {AA, AB};
  const int smode[2] = {aj, bj};
  std::vector<Fam> F;
  std::vector<std::unique_ptr<Group>> inter;  // intermediates of this step
  auto fam = [&](int out, int out_base, int count, const Group* src, int src_base, bool trans, const Mat4& s,
                 int pi, double coef = 1.0, std::vector<double> cv = {}) {
    if (count <= 0 || site::zero(s)) return;
    Fam f;
    f.out = out;
    f.out_base = out_base;
    f.count = count;
    f.src = src;
    f.src_base = src_base;
    f.trans = trans;
    f.s = s;
    f.pi = pi;
    f.coef = coef;
    f.cv = std::move(cv);
    F.push_back(std::move(f));
  };
  const Group* XG = X.g.data();
  // pi of a product: left growth -> parity of the site factor; right -> parity of the block factor
  auto PI = [&](int site_par, int blk_par) { return left ? site_par : blk_par; };

  // offsets of the "new" parts inside Z member lists
  const int nA = left ? X.g[G_AAA].n() : 0, nB = left ? X.g[G_ABB].n() : 0, nAB = left ? X.g[G_AAB].n() : 0;
  const int nB0 = left ? X.g[G_B0].n() : 0, nBab = left ? X.g[G_BAB].n() : 0, nBba = left ? X.g[G_BBA].n() : 0;
  const int oldoff_ca = left ? 0 : 1;

  // a+_p
  fam(G_CA, oldoff_ca, nXa, &XG[G_CA], 0, false, I4, PI(0, 1));
  fam(G_CB, oldoff_ca, nXb, &XG[G_CB], 0, false, I4, PI(0, 1));
  fam(G_CA, left ? nXa : 0, 1, nullptr, 0, false, CA, PI(1, 0));
  fam(G_CB, left ? nXb : 0, 1, nullptr, 0, false, CB, PI(1, 0));
  // inherited two-index operators: X-op (x) I
  {
    const int gids[6] = {G_AAA, G_AAB, G_ABB, G_B0, G_BAB, G_BBA};
    for (int gid : gids) {
      int nold = X.g[gid].n();
      int base = left ? 0 : Z.g[gid].n() - nold;
      fam(gid, base, nold, &XG[gid], 0, false, I4, 0);
    }
  }
  // new pair operators.  Left: block mode p < site mode; product (block op).(site op).
  // Right: site mode < block mode; product (site op).(block op).
  if (left) {
    // A_{p,aj} = a+_p a+_aj
    fam(G_AAA, nA, nXa, &XG[G_CA], 0, false, CA, 1);
    fam(G_ABB, nB, nXb, &XG[G_CB], 0, false, CB, 1);
    fam(G_AAB, nAB, nXa, &XG[G_CA], 0, false, CB, 1);
    fam(G_AAB, nAB + nXa, nXb, &XG[G_CB], 0, false, CA, 1);
    fam(G_AAB, nAB + nXa + nXb, 1, nullptr, 0, false, mul(CA, CB), 0);
    // B_{p,s}: a+_p a_site ; a+_site a_p = -a_p a+_site
    for (int sp = 0; sp < 2; ++sp) {
      const Group* cg = &XG[sp ? G_CB : G_CA];
      int nx = sp ? nXb : nXa;
      int o = nB0 + (sp ? 2 * nXa + 1 : 0);
      fam(G_B0, o, nx, cg, 0, false, ANN[sp], 1);
      fam(G_B0, o + nx, nx, cg, 0, true, CRE[sp], 1, -1.0);
      fam(G_B0, o + 2 * nx, 1, nullptr, 0, false, mul(CRE[sp], ANN[sp]), 0);
    }
    fam(G_BAB, nBab, nXa, &XG[G_CA], 0, false, AB, 1);
    fam(G_BAB, nBab + nXa, nXb, &XG[G_CB], 0, true, CA, 1, -1.0);
    fam(G_BAB, nBab + nXa + nXb, 1, nullptr, 0, false, mul(CA, AB), 0);
    fam(G_BBA, nBba, nXb, &XG[G_CB], 0, false, AA, 1);
    fam(G_BBA, nBba + nXb, nXa, &XG[G_CA], 0, true, CB, 1, -1.0);
    fam(G_BBA, nBba + nXb + nXa, 1, nullptr, 0, false, mul(CB, AA), 0);
  } else {
    // A_{aj,q} = a+_aj a+_q
    fam(G_AAA, 0, nXa, &XG[G_CA], 0, false, CA, 1);
    fam(G_ABB, 0, nXb, &XG[G_CB], 0, false, CB, 1);
    fam(G_AAB, 0, nXb, &XG[G_CB], 0, false, CA, 1);
    fam(G_AAB, nXb, nXa, &XG[G_CA], 0, false, CB, 1);
    fam(G_AAB, nXa + nXb, 1, nullptr, 0, false, mul(CA, CB), 0);
    for (int sp = 0; sp < 2; ++sp) {
      const Group* cg = &XG[sp ? G_CB : G_CA];
      int nx = sp ? nXb : nXa;
      int o = sp ? 2 * nXa + 1 : 0;
      // B_{site,s} = a+_site a_s
      fam(G_B0, o, nx, cg, 0, true, CRE[sp], 1);
      // B_{p,site} = a+_p a_site = -a_site a+_p
      fam(G_B0, o + nx, nx, cg, 0, false, ANN[sp], 1, -1.0);
      fam(G_B0, o + 2 * nx, 1, nullptr, 0, false, mul(CRE[sp], ANN[sp]), 0);
    }
    fam(G_BAB, 0, nXb, &XG[G_CB], 0, true, CA, 1);
    fam(G_BAB, nXb, nXa, &XG[G_CA], 0, false, AB, 1, -1.0);
    fam(G_BAB, nXb + nXa, 1, nullptr, 0, false, mul(CA, AB), 0);
    fam(G_BBA, 0, nXa, &XG[G_CA], 0, true, CB, 1);
    fam(G_BBA, nXa, nXb, &XG[G_CB], 0, false, AA, 1, -1.0);
    fam(G_BBA, nXa + nXb, 1, nullptr, 0, false, mul(CB, AA), 0);
  }

  // ---- helpers for intermediates (linear combinations of X groups)
  auto cre_group = [&](int sp) -> const Group& { return XG[sp ? G_CB : G_CA]; };
  auto a_group = [&](int s1, int s2) -> const Group& {
    return XG[(s1 == 0 && s2 == 0) ? G_AAA : ((s1 == 1 && s2 == 1) ? G_ABB : G_AAB)];
  };
  // B group holding a+_q a_t with the spins needed by Q_{pr} = sum <pq||rt> B_qt
  auto q_source = [&](int sp, int sr) -> const Group& {
    if (sp == sr) return XG[G_B0];
    return XG[sp == 0 ? G_BBA : G_BAB];
  };
  auto coefQ = [&](const Group& src, int p, int r) {
    std::vector<double> c(src.n(), 0.0);
    for (int m = 0; m < src.n(); ++m) {
      const OpKey& k = src.names[m];
      if (k.kind == 'B') c[m] = I.w(p, k.p, r, k.q);
    }
    return c;
  };
  auto coefW = [&](const Group& src, int p, int q) {  // Y_pq = sum_{s<r} <pq||sr> A_sr
    std::vector<double> c(src.n(), 0.0);
    for (int m = 0; m < src.n(); ++m) {
      const OpKey& k = src.names[m];
      c[m] = I.w(p, q, k.p, k.q);
    }
    return c;
  };
  auto make_inter = [&](const Group& src, std::vector<std::vector<double>> rows) -> const Group* {
    std::vector<OpKey> nm(rows.size(), OpKey{'X', -1, -1});
    inter.push_back(combine(src, rows, nm, true));
    return inter.back().get();
  };
  auto nonzero = [](const std::vector<double>& v) {
    for (double x : v)
      if (x != 0.0) return true;
    return false;
  };

  // S^site_p monomials: a_q (1/2 t_pq), a+_q a_b a_a (<pq||ab>)
  const Mat4 SMON[4] = {AA, AB, mul(CA, mul(AB, AA)), mul(CB, mul(AB, AA))};
  auto smon_coef = [&](int p, int m) {
    switch (m) {
      case 0: return 0.5 * I.t(p, aj);
      case 1: return 0.5 * I.t(p, bj);
      case 2: return I.w(p, aj, aj, bj);
      default: return I.w(p, bj, aj, bj);
    }
  };
  const int SMON_PSPIN[4] = {0, 1, 1, 0};  // spin of p for which monomial m can be nonzero

  // ---- S_p (p external to Z), per spin group
  for (int sp = 0; sp < 2; ++sp) {
    const int gid = sp ? G_SB : G_SA;
    const std::vector<int>& ext = sp ? Z.ext_b : Z.ext_a;
    const int n = (int)ext.size();
    if (n == 0) continue;
    const int xbase = sp ? sb_base : sa_base;
    // S^X_p (x) I  (left)  /  I (x) S^X_p  (right)
    fam(gid, 0, n, &XG[gid], xbase, false, I4, PI(0, 1));
    // site S_p monomials with identity on the block
    for (int m = 0; m < 4; ++m) {
      std::vector<double> cv(n);
      for (int i = 0; i < n; ++i) cv[i] = smon_coef(ext[i], m);
      if (nonzero(cv)) fam(gid, 0, n, nullptr, 0, false, SMON[m], PI(1, 0), 1.0, cv);
    }
    // Q^X_{pr} with r on the site:
    //   left:  Q^X_pr . a_r              right: a_r . Q^X_pr
    for (int rs = 0; rs < 2; ++rs) {
      const Group& src = q_source(sp, rs);
      std::vector<std::vector<double>> rows;
      for (int i = 0; i < n; ++i) rows.push_back(coefQ(src, ext[i], smode[rs]));
      const Group* Q = make_inter(src, rows);
      fam(gid, 0, n, Q, 0, false, ANN[rs], PI(1, 0));
    }
    // block single a_s times site a+_q a_t:
    //   left:  sum_{q,t} (sum_{s in X} <pq||st> a_s) . a+_q a_t
    //   right: sum_{q,t} a+_q a_t . (sum_{r in X} <pq||rt> a_r)
    for (int qs = 0; qs < 2; ++qs)
      for (int ts = 0; ts < 2; ++ts) {
        int ss = (qs == ts) ? sp : (sp == ts ? qs : -1);
        if (ss < 0) continue;
        const Group& src = cre_group(ss);
        std::vector<std::vector<double>> rows;
        for (int i = 0; i < n; ++i) {
          std::vector<double> c(src.n());
          for (int m = 0; m < src.n(); ++m) {
            int s = src.names[m].p;
            c[m] = left ? I.w(ext[i], smode[qs], s, smode[ts]) : I.w(ext[i], smode[qs], s, smode[ts]);
          }
          rows.push_back(c);
        }
        const Group* U = make_inter(src, rows);
        fam(gid, 0, n, U, 0, true, mul(CRE[qs], ANN[ts]), PI(0, 1));
      }
    // a+ (block) combined with the site pair annihilator a_b a_a:
    //   left:  (sum_q <pq||ab> a+_q) . a_b a_a     right: a_b a_a . (sum_q <pq||ab> a+_q)
    {
      const Group& src = cre_group(1 - sp);
      std::vector<std::vector<double>> rows;
      for (int i = 0; i < n; ++i) {
        std::vector<double> c(src.n());
        for (int m = 0; m < src.n(); ++m) c[m] = I.w(ext[i], src.names[m].p, aj, bj);
        rows.push_back(c);
      }
      const Group* V = make_inter(src, rows);
      fam(gid, 0, n, V, 0, false, mul(AB, AA), PI(0, 1));
    }
    // P^X_{pq} with q on the site (P = Y^T):
    //   left: P^X_pq . a+_q      right: a+_q . P^X_pq
    for (int qs = 0; qs < 2; ++qs) {
      const Group& src = a_group(sp, qs);
      std::vector<std::vector<double>> rows;
      for (int i = 0; i < n; ++i) rows.push_back(coefW(src, ext[i], smode[qs]));
      const Group* W = make_inter(src, rows);
      fam(gid, 0, n, W, 0, true, CRE[qs], PI(1, 0));
    }
  }

  // ---- H (normal operators on the site side)
  fam(G_H, 0, 1, &XG[G_H], 0, false, I4, 0);
  {
    Mat4 Hs{};
    for (int ps = 0; ps < 2; ++ps)
      for (int qs = 0; qs < 2; ++qs) {
        double tv = I.t(smode[ps], smode[qs]);
        if (tv != 0.0) {
          Mat4 m = mul(CRE[ps], ANN[qs]);
          for (int i = 0; i < 16; ++i) Hs[i] += tv * m[i];
        }
      }
    Mat4 m2 = mul(mul(CA, CB), mul(AB, AA));
    double wv = I.w(aj, bj, aj, bj);
    for (int i = 0; i < 16; ++i) Hs[i] += wv * m2[i];
    fam(G_H, 0, 1, nullptr, 0, false, Hs, 0);
  }
  // block a+_p with the site's S_p monomials:
  //   left:  sum_p [a+_p . S^s_p - a_p . S^s_p^T]
  //   right: sum_p [-S^s_p . a+_p + S^s_p^T . a_p]
  for (int m = 0; m < 4; ++m) {
    int ps = SMON_PSPIN[m];
    const Group& src = cre_group(ps);
    if (src.n() == 0) continue;
    std::vector<double> c(src.n());
    for (int i = 0; i < src.n(); ++i) c[i] = smon_coef(src.names[i].p, m);
    if (!nonzero(c)) continue;
    const Group* Y = make_inter(src, {c});
    fam(G_H, 0, 1, Y, 0, false, SMON[m], 1, left ? 1.0 : -1.0);
    fam(G_H, 0, 1, Y, 0, true, tr(SMON[m]), 1, left ? -1.0 : 1.0);
  }
  // site a+_p with the block's S_p:
  //   left:  sum_{p on site} [-S^X_p . a+_p + S^X_p^T . a_p]
  //   right: sum_{p on site} [a+_p . S^X_p - a_p . S^X_p^T]
  for (int ps = 0; ps < 2; ++ps) {
    const int gid = ps ? G_SB : G_SA;
    const int mem = left ? 0 : X.g[gid].n() - 1;
    fam(G_H, 0, 1, &XG[gid], mem, false, CRE[ps], 1, left ? -1.0 : 1.0);
    fam(G_H, 0, 1, &XG[gid], mem, true, ANN[ps], 1, left ? 1.0 : -1.0);
  }
  // P^X_{ab} with A^site_{ab} + h.c.   (P^X = W^T)
  {
    const Group& src = a_group(0, 1);
    if (src.n() > 0) {
      const Group* W = make_inter(src, {coefW(src, aj, bj)});
      fam(G_H, 0, 1, W, 0, true, mul(CA, CB), 0);
      fam(G_H, 0, 1, W, 0, false, tr(mul(CA, CB)), 0);
    }
  }
  // Q^X_{ps} with B^site_{ps}
  for (int ps = 0; ps < 2; ++ps)
    for (int ss = 0; ss < 2; ++ss) {
      const Group& src = q_source(ps, ss);
      if (src.n() == 0) continue;
      const Group* Q = make_inter(src, {coefQ(src, smode[ps], smode[ss])});
      fam(G_H, 0, 1, Q, 0, false, mul(CRE[ps], ANN[ss]), 0);
    }

  // ---- execute families (stream order covers the intermediates' launches)
  const Basis& XB = X.basis;
  const Basis& ZB = Z.basis;
  // coefficient vectors to the device
  std::vector<double> cvall;
  std::vector<int64_t> cvoff(F.size(), -1);
  for (size_t f = 0; f < F.size(); ++f)
    if (!F[f].cv.empty()) {
      cvoff[f] = (int64_t)cvall.size();
      cvall.insert(cvall.end(), F[f].cv.begin(), F[f].cv.end());
    }
  double* dcv = nullptr;
  int cvbuf = -1;
  if (!cvall.empty()) {  // read by launches all through the step: not in the ring
    dcv = (double*)step_arena.take(cvall.size() * sizeof(double));
    dev_h2d(dcv, cvall.data(), cvall.size() * sizeof(double));
    cvbuf = tab.add(dcv);
  }
  double* T = nullptr;
  size_t Tcap = 0;
  int Tbuf = tab.add(nullptr);

  for (size_t fi = 0; fi < F.size(); ++fi) {
    const Fam& f = F[fi];
    const Group& out = Z.g[f.out];
    if (out.lay.size == 0) continue;
    // T entries: key (n, z-sector) -> offset, block bra, block ket
    struct TE {
      int64_t off;
      int xbra, xket, a;
    };
    std::map<std::pair<int, int>, TE> tmap;
    int64_t tstride = 0;
    if (f.src) {
      const Layout& sl = f.src->lay;
      for (int xk = 0; xk < XB.nsec(); ++xk) {
        int xbra;
        if (eff_block(sl, f.trans, xk, &xbra) < 0) continue;
        for (int n = 0; n < 4; ++n) {
          bool col = false;
          for (int n1 = 0; n1 < 4; ++n1) col |= f.s[n1 * 4 + n] != 0.0;
          if (!col) continue;
          auto it = left ? A.by_left.find({xk, n}) : A.by_right.find({xk, n});
          if (it == (left ? A.by_left.end() : A.by_right.end())) continue;
          int a = it->second;
          int zs = left ? A.ir[a] : A.il[a];
          tmap[{n, zs}] = TE{tstride, xbra, xk, a};
          tstride += (int64_t)XB.dim[xbra] * ZB.dim[zs];
        }
      }
      if (tstride == 0) continue;
    }
    int chunk = f.count;
    if (f.src) {
      size_t per = (size_t)tstride * sizeof(double);
      chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)f.count, scratch_budget / per));
      size_t need = per * (size_t)chunk;
      if (need > Tcap) {  // every T block is written by phase 1 before phase 2 reads it
        T = (double*)step_arena.take(need);
        Tcap = need;
        tab.set(Tbuf, T);
      }
    }
    for (int c0 = 0; c0 < f.count; c0 += chunk) {
      const int nb = std::min(chunk, f.count - c0);
      GemmList p1, p2;
      if (f.src) {
        const Layout& sl = f.src->lay;
        const int64_t ss = f.src->stride();
        for (auto& kv : tmap) {
          const TE& e = kv.second;
          const int zs = kv.first.second;
          const int sb = f.trans ? sl.by_bra[e.xket] : sl.by_ket[e.xket];
          const int dxb = XB.dim[e.xbra], dxk = XB.dim[e.xket], dz = ZB.dim[zs];
          const int ld_src = f.trans ? dxb : dxk;
          p1.begin(dxb, dz, nb, Tbuf, e.off, dz, tstride, false);
          GContrib c = make_contrib(dxk, f.trans ? GF_TRANS_A : 0, f.src->buf,
                                    (int64_t)(f.src_base + c0) * ss + sl.off[sb], ld_src, A.buf, A.off[e.a],
                                    left ? dz : dxk, 1.0);
          if (!left) c.flags |= GF_TRANS_B;
          c.a_bstride = ss;
          p1.add(c);
          p1.end();
        }
      }
      // phase 2: output blocks of Z
      const Layout& ol = out.lay;
      for (int ob = 0; ob < ol.nblk(); ++ob) {
        const int zb = ol.bra[ob], zk = ol.ket[ob];
        p2.begin(ZB.dim[zb], ZB.dim[zk], nb, out.buf, (int64_t)(f.out_base + c0) * out.stride() + ol.off[ob],
                 ZB.dim[zk], out.stride(), true);
        for (int n1 = 0; n1 < 4; ++n1)
          for (int n = 0; n < 4; ++n) {
            const double sv = f.s[n1 * 4 + n];
            if (sv == 0.0) continue;
            // blocks of A touching the ket (zk, n) and the bra (zb, n1)
            auto ita = left ? A.by_right.find({zk, n}) : A.by_left.find({zk, n});
            auto itb = left ? A.by_right.find({zb, n1}) : A.by_left.find({zb, n1});
            auto endm = left ? A.by_right.end() : A.by_left.end();
            if (ita == endm || itb == endm) continue;
            const int a = ita->second, ab = itb->second;
            const int xk = left ? A.il[a] : A.ir[a];
            const int xbra = left ? A.il[ab] : A.ir[ab];
            double alpha = f.coef * sv;
            if (f.pi) {
              int ne = left ? XB.qn[xk].n() : site::nelec(n);
              if (ne & 1) alpha = -alpha;
            }
            const int dxb = XB.dim[xbra];
            GContrib c{};
            if (left) {
              // O(zb,zk) += alpha A(xbra,n1,zb)^T . T(xbra,n,zk)
              c = make_contrib(dxb, GF_TRANS_A, A.buf, A.off[ab], ZB.dim[zb], 0, 0, ZB.dim[zk], alpha);
            } else {
              // O(zb,zk) += alpha A(zb,n1,xbra) . T(xbra,n,zk)
              c = make_contrib(dxb, 0, A.buf, A.off[ab], dxb, 0, 0, ZB.dim[zk], alpha);
            }
            if (f.src) {
              auto it = tmap.find({n, zk});
              if (it == tmap.end() || it->second.xbra != xbra) continue;
              c.b_buf = Tbuf;
              c.b_off = it->second.off;
              c.b_bstride = tstride;
            } else {
              if (xbra != xk) continue;  // identity on the block
              c.b_buf = A.buf;
              c.b_off = A.off[a];
              if (left) {
                c.ldb = ZB.dim[zk];
              } else {
                c.flags |= GF_TRANS_B;
                c.ldb = XB.dim[xk];
              }
            }
            if (cvoff[fi] >= 0) {
              c.s_buf = cvbuf;
              c.s_off = cvoff[fi] + c0;
              c.s_bstride = 1;
            }
            p2.add(c);
          }
        p2.end();
      }
      run(p1);
      run(p2);
    }
  }
  dev_sync(stream);
  tab.set(Tbuf, nullptr);
  if (cvbuf >= 0) tab.set(cvbuf, nullptr);
  for (auto& g : inter) {
    tab.set(g->buf, nullptr);
    g->free_dev();
  }
  step_arena.reset();
  return Zp;
}

}  // namespace dmrg
