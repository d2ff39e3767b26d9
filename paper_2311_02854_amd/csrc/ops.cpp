// Build one bond's operators on the GPU and plan sigma = H psi.
//
// The two-dot Hamiltonian (Eq. totoalH) is written as a sum of triples
// O^L . O^D . O^R over the left block L (sites < k), the two dots D = C1 u C2
// (sites k, k+1, exact 16x16 operators) and the right block R (sites > k+1).
// Grouped by where the (up to four) spin-orbital indices of each monomial of
// Eq. (Hsq) live, with normal operators on L and complementary ones on R:
//   H^L, H^D, H^R                          (4,0,0) (0,4,0) (0,0,4)
//   S^L_d a+_d, a+_p S^D_p                 (3,1,0) (1,3,0)
//   S^L_r a+_r, a+_p S^R_p                 (3,0,1) (1,0,3)
//   S^D_r a+_r, a+_d S^R_d                 (0,3,1) (0,1,3)
//   P^L A^D + Q^L B^D, A^D P^R + B^D Q^R   (2,2,0) (0,2,2)
//   A^L P^R + B^L Q^R                      (2,0,2)   <- O(K^2) terms, the bulk
//   P^L_dr a+_d a+_r ..., a+_p a+_d P^R_pd ..., a_s Q^D_rs a+_r ...   (2,1,1) (1,1,2) (1,2,1)
// ("+ h.c." throughout).  Every triple acts on |l c1 c2 r> with the sign
// zeta = (-1)^(pi_D N_l + pi_R (N_l + N_c1 + N_c2)) (Eq. Sigma).
// Per psi block the contraction is the paper's eight-batch scheme reduced to
// two batches (site factors are scalars, Sec. 2.2): X = psi . (O^R)^T
// (Eq. sigmablk56) and sigma += c zeta D O^L . X (Eqs. sigmablk78, sigmablk).
#include "ops.h"

#include <algorithm>
#include <atomic>
#include <numeric>
#include <cmath>
#include <map>
#include <set>

namespace dmrg {

namespace dot {
Mat16 I16() {
  Mat16 m{};
  for (int i = 0; i < 16; ++i) m[i * 16 + i] = 1.0;
  return m;
}
Mat16 kron(const Mat4& a, const Mat4& b) {
  Mat16 m{};
  for (int i1 = 0; i1 < 4; ++i1)
    for (int j1 = 0; j1 < 4; ++j1)
      for (int i2 = 0; i2 < 4; ++i2)
        for (int j2 = 0; j2 < 4; ++j2) m[(i1 * 4 + i2) * 16 + (j1 * 4 + j2)] = a[i1 * 4 + j1] * b[i2 * 4 + j2];
  return m;
}
Mat16 mul(const Mat16& a, const Mat16& b) {
  Mat16 m{};
  for (int i = 0; i < 16; ++i)
    for (int k = 0; k < 16; ++k) {
      double x = a[i * 16 + k];
      if (x == 0.0) continue;
      for (int j = 0; j < 16; ++j) m[i * 16 + j] += x * b[k * 16 + j];
    }
  return m;
}
Mat16 tr(const Mat16& a) {
  Mat16 m{};
  for (int i = 0; i < 16; ++i)
    for (int j = 0; j < 16; ++j) m[i * 16 + j] = a[j * 16 + i];
  return m;
}
Mat16 add(const Mat16& a, const Mat16& b, double s) {
  Mat16 m = a;
  for (int i = 0; i < 256; ++i) m[i] += s * b[i];
  return m;
}
bool zero(const Mat16& a) {
  for (double x : a)
    if (x != 0.0) return false;
  return true;
}
// local dot modes: 0 = alpha of C1, 1 = beta of C1, 2 = alpha of C2, 3 = beta of C2
Mat16 cre(int d) {
  Mat4 par{};
  par[0] = 1;
  par[5] = -1;
  par[10] = -1;
  par[15] = 1;
  if (d < 2) return kron(site::cre(d), site::I());
  return kron(par, site::cre(d - 2));  // Jordan-Wigner string through C1
}
Mat16 ann(int d) { return tr(cre(d)); }
int nelec(int e) { return SITE_QN[e / 4].n() + SITE_QN[e % 4].n(); }
}  // namespace dot

void Ops::begin_call(void* stream) {
  if (used && stream != last_stream && order_ev) stream_wait(stream, order_ev);
}

void Ops::end_call(void* stream) {
  if (!order_ev) order_ev = ev_create();
  ev_record(order_ev, stream);
  last_stream = stream;
  used = true;
}

Ops::~Ops() {
  launches.clear();
  for (void* e : events) ev_destroy(e);
  ev_destroy(order_ev);
  if (L) L->free_dev();
  if (R) R->free_dev();
  for (auto& g : extra) g->free_dev();
  dev_free(X[0]);
  dev_free(X[1]);
  dev_free(partial);
  dev_free(perm_seg);
  dev_free(psi_perm);
  dev_free(psi_perm32);
  dev_free(X32[0]);
  dev_free(X32[1]);
  dev_free(psi32);
  dev_free(mlp_blk);
  dev_free(mlp_stat);
  dev_free(mlp_part);
  dev_free(mlp_scales);
  dev_free(mlp_w);
}

namespace {

std::unique_ptr<SiteTensor> upload_site(int j, const std::vector<std::vector<QN>>& labels,
                                        const std::vector<std::vector<int>>& dims, const int64_t* blk_off,
                                        int64_t& bcount, const double* data) {
  auto A = std::make_unique<SiteTensor>();
  std::vector<double> host;
  const auto& lq = labels[j];
  const auto& rq = labels[j + 1];
  for (int il = 0; il < (int)lq.size(); ++il)
    for (int n = 0; n < 4; ++n) {
      QN q = lq[il] + SITE_QN[n];
      int ir = -1;
      for (int t = 0; t < (int)rq.size(); ++t)
        if (rq[t] == q) ir = t;
      if (ir < 0) continue;
      int64_t src = blk_off[bcount++];
      int64_t cnt = (int64_t)dims[j][il] * dims[j + 1][ir];
      A->off.push_back((int64_t)host.size());
      A->il.push_back(il);
      A->n.push_back(n);
      A->ir.push_back(ir);
      A->by_left[{il, n}] = (int)A->il.size() - 1;
      A->by_right[{ir, n}] = (int)A->il.size() - 1;
      host.insert(host.end(), data + src, data + src + cnt);
    }
  A->dev = (double*)dev_alloc(std::max<size_t>(1, host.size()) * sizeof(double));
  dev_h2d(A->dev, host.data(), host.size() * sizeof(double));
  return A;
}

Basis make_basis(const std::vector<QN>& labels, const std::vector<int>& dims, bool left, int Na, int Nb) {
  Basis B;
  for (size_t i = 0; i < labels.size(); ++i) {
    B.qn.push_back(left ? labels[i] : QN(Na - labels[i].a, Nb - labels[i].b));
    B.dim.push_back(dims[i]);
  }
  B.finish();
  return B;
}

// member list builder that records run bases
struct Names {
  std::vector<OpKey> v;
  int add_run(const std::vector<OpKey>& r) {
    int b = (int)v.size();
    v.insert(v.end(), r.begin(), r.end());
    return b;
  }
};

}  // namespace

// ----------------------------------------------------------------------------
std::unique_ptr<Ops> build_ops(const Integrals& I, int K, int Na, int Nb, int bond, const int* nsec,
                               const int* sec_qn, const int* sec_dim, const int64_t* blk_off,
                               const double* data, void* stream, const BuildOptions& opt) {
  const double t0 = wall_seconds();
  DMRG_CHECK(K >= 2 && bond >= 0 && bond <= K - 2, DMRG_EINVAL, "bond must satisfy 0 <= bond <= K-2");
  DMRG_CHECK(Na >= 0 && Nb >= 0 && Na <= K && Nb <= K, DMRG_EINVAL, "electron numbers out of range");
  auto ops = std::make_unique<Ops>();
  Ops& O = *ops;
  static std::atomic<uint64_t> serial_counter{0};
  O.serial = ++serial_counter;
  O.K = K;
  O.Na = Na;
  O.Nb = Nb;
  O.bond = bond;
  O.ints = I;
  O.ecore = I.ecore;
  O.tab = std::make_unique<DevTable>();
  DevTable& tab = *O.tab;
  // sectors
  std::vector<std::vector<QN>> labels(K + 1);
  std::vector<std::vector<int>> dims(K + 1);
  {
    int64_t pos = 0;
    for (int b = 0; b <= K; ++b) {
      DMRG_CHECK(nsec[b] >= 1, DMRG_ESHAPE, "every bond needs at least one sector");
      for (int i = 0; i < nsec[b]; ++i, ++pos) {
        QN q(sec_qn[2 * pos], sec_qn[2 * pos + 1]);
        DMRG_CHECK(sec_dim[pos] > 0, DMRG_ESHAPE, "sector dimensions must be positive");
        for (auto& o : labels[b]) DMRG_CHECK(!(o == q), DMRG_ESHAPE, "duplicate sector at a bond");
        labels[b].push_back(q);
        dims[b].push_back(sec_dim[pos]);
      }
    }
    DMRG_CHECK(labels[0].size() == 1 && labels[0][0] == QN(0, 0) && dims[0][0] == 1, DMRG_ESHAPE,
               "bond 0 must hold the single vacuum sector");
    DMRG_CHECK(labels[K].size() == 1 && labels[K][0] == QN(Na, Nb) && dims[K][0] == 1, DMRG_ESHAPE,
               "bond K must hold the single target sector");
  }
  Builder bld(I, tab, stream, Na, Nb);
  bld.scratch_budget = opt.t_budget;
  // site tensors are stored for j < bond then j > bond+1, ascending
  std::vector<int64_t> first_blk(K, -1);
  {
    int64_t bc = 0;
    for (int j = 0; j < K; ++j) {
      if (j == bond || j == bond + 1) continue;
      first_blk[j] = bc;
      const auto& lq = labels[j];
      for (int il = 0; il < (int)lq.size(); ++il)
        for (int n = 0; n < 4; ++n) {
          QN q = lq[il] + SITE_QN[n];
          for (auto& r : labels[j + 1])
            if (r == q) ++bc;
        }
    }
  }
  // ---- grow the left block over sites 0..bond-1
  auto Lblk = bld.vacuum(true);
  for (int j = 0; j < bond; ++j) {
    int64_t bc = first_blk[j];
    auto A = upload_site(j, labels, dims, blk_off, bc, data);
    A->buf = tab.add(A->dev);
    auto Z = bld.grow(*Lblk, j, *A, make_basis(labels[j + 1], dims[j + 1], true, Na, Nb), j == bond - 1);
    dev_sync(stream);
    tab.set(A->buf, nullptr);
    Lblk = std::move(Z);
  }
  // ---- grow the right block over sites K-1..bond+2
  auto Rblk = bld.vacuum(false);
  for (int j = K - 1; j > bond + 1; --j) {
    int64_t bc = first_blk[j];
    auto A = upload_site(j, labels, dims, blk_off, bc, data);
    A->buf = tab.add(A->dev);
    auto Z = bld.grow(*Rblk, j, *A, make_basis(labels[j], dims[j], false, Na, Nb), j == bond + 2);
    dev_sync(stream);
    tab.set(A->buf, nullptr);
    Rblk = std::move(Z);
  }
  O.Lb = Lblk->basis;
  O.Rb = Rblk->basis;
  O.Llabel = labels[bond];
  O.Rlabel = labels[bond + 2];
  O.L = std::move(Lblk);
  O.R = std::move(Rblk);
  const Block& L = *O.L;
  const Block& R = *O.R;
  const int k = bond;
  auto dmode = [&](int d) { return 2 * k + d; };
  auto dspin = [](int d) { return d & 1; };

  // ---- psi layout
  {
    const int nL = O.Lb.nsec(), nR = O.Rb.nsec();
    O.blk_index.assign((size_t)nL * 16 * nR, -1);
    for (int il = 0; il < nL; ++il)
      for (int n1 = 0; n1 < 4; ++n1)
        for (int n2 = 0; n2 < 4; ++n2) {
          QN q = O.Llabel[il] + SITE_QN[n1] + SITE_QN[n2];
          int ir = -1;
          for (int t = 0; t < nR; ++t)
            if (O.Rlabel[t] == q) ir = t;
          if (ir < 0) continue;
          PsiBlk b{il, n1 * 4 + n2, ir, O.Lb.dim[il], O.Rb.dim[ir], O.npsi};
          O.blk_index[((size_t)il * 16 + b.e) * nR + ir] = (int)O.blocks.size();
          O.blocks.push_back(b);
          O.npsi += (int64_t)b.dl * b.dr;
        }
    DMRG_CHECK(O.npsi > 0, DMRG_ESHAPE, "the two-dot space is empty");
  }

  // ---- complementary operators on R: Y^R_pq = sum_{s<r in R} <pq||sr> A_sr (P^R = Y^T)
  //      and Q^R_ps = sum_{q,r in R} <pq||sr> B_qr, for p, q, s in L u D
  auto coefW = [&](const Group& src, int p, int q) {
    std::vector<double> c(src.n());
    for (int m = 0; m < src.n(); ++m) c[m] = I.w(p, q, src.names[m].p, src.names[m].q);
    return c;
  };
  auto coefQ = [&](const Group& src, int p, int s) {
    std::vector<double> c(src.n());
    for (int m = 0; m < src.n(); ++m) c[m] = I.w(p, src.names[m].p, s, src.names[m].q);
    return c;
  };
  auto a_gid = [](int s1, int s2) { return (s1 == 0 && s2 == 0) ? G_AAA : ((s1 == 1 && s2 == 1) ? G_ABB : G_AAB); };
  auto y_cls = [](int s1, int s2) { return (s1 == 0 && s2 == 0) ? 0 : ((s1 == 1 && s2 == 1) ? 2 : 1); };
  auto q_cls = [](int sp, int ss) { return sp == ss ? 0 : (sp == 0 ? 1 : 2); };  // Q0, Qab, Qba
  auto q_src_gid = [](int sp, int ss) { return sp == ss ? G_B0 : (sp == 0 ? G_BBA : G_BAB); };
  const int LQG[3] = {G_B0, G_BAB, G_BBA};
  const int LAG[3] = {G_AAA, G_AAB, G_ABB};
  const auto& Lca = L.g[G_CA].names;
  const auto& Lcb = L.g[G_CB].names;
  const std::vector<OpKey>* Lc[2] = {&Lca, &Lcb};

  Names Yn[3], Qn[3];
  int yb[4][2], qb1[4][2], qb2[4][2], ydd[4][4], qdd[4][4];
  for (int c = 0; c < 3; ++c) {
    for (auto& kk : L.g[LAG[c]].names) Yn[c].v.push_back({'Y', kk.p, kk.q});
    for (auto& kk : L.g[LQG[c]].names) Qn[c].v.push_back({'Q', kk.p, kk.q});
  }
  for (int d = 0; d < 4; ++d)
    for (int s = 0; s < 2; ++s) {
      std::vector<OpKey> ry, rq1, rq2;
      for (auto& kk : *Lc[s]) {
        ry.push_back({'Y', kk.p, dmode(d)});
        rq1.push_back({'Q', kk.p, dmode(d)});
        rq2.push_back({'Q', dmode(d), kk.p});
      }
      yb[d][s] = Yn[y_cls(s, dspin(d))].add_run(ry);
      qb1[d][s] = Qn[q_cls(s, dspin(d))].add_run(rq1);
      qb2[d][s] = Qn[q_cls(dspin(d), s)].add_run(rq2);
    }
  for (int d = 0; d < 4; ++d)
    for (int e = 0; e < 4; ++e) {
      ydd[d][e] = -1;
      if (d < e) ydd[d][e] = Yn[y_cls(dspin(d), dspin(e))].add_run({{'Y', dmode(d), dmode(e)}});
      qdd[d][e] = Qn[q_cls(dspin(d), dspin(e))].add_run({{'Q', dmode(d), dmode(e)}});
    }
  const Group* YR[3];
  const Group* QR[3];
  for (int c = 0; c < 3; ++c) {
    // Y class c pairs (p<q) with spins matching the A group of R
    const int sp1 = (c == 2) ? 1 : 0;
    (void)sp1;
    std::vector<std::vector<double>> rows;
    const Group* srcA = nullptr;
    for (auto& kk : Yn[c].v) {
      const Group& src = R.g[a_gid(kk.p & 1, kk.q & 1)];
      srcA = &src;
      rows.push_back(coefW(src, kk.p, kk.q));
    }
    if (!srcA) srcA = &R.g[LAG[c]];
    O.extra.push_back(bld.combine(*srcA, rows, Yn[c].v));
    YR[c] = O.extra.back().get();
    rows.clear();
    const Group* srcQ = nullptr;
    for (auto& kk : Qn[c].v) {
      const Group& src = R.g[q_src_gid(kk.p & 1, kk.q & 1)];
      srcQ = &src;
      rows.push_back(coefQ(src, kk.p, kk.q));
    }
    if (!srcQ) srcQ = &R.g[c == 0 ? G_B0 : (c == 1 ? G_BBA : G_BAB)];
    O.extra.push_back(bld.combine(*srcQ, rows, Qn[c].v));
    QR[c] = O.extra.back().get();
  }
  // the normal two-index operators of R are no longer needed
  for (int gid : {G_AAA, G_AAB, G_ABB, G_B0, G_BAB, G_BBA}) {
    tab.set(O.R->g[gid].buf, nullptr);
    O.R->g[gid].free_dev();
  }

  // ---- dot operators
  using namespace dot;
  const Mat16 Id = I16();
  Mat16 Dc[4], Da[4];
  for (int d = 0; d < 4; ++d) {
    Dc[d] = cre(d);
    Da[d] = ann(d);
  }
  Mat16 HD{};
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) {
      double tv = I.t(dmode(p), dmode(q));
      if (tv != 0.0) HD = add(HD, mul(Dc[p], Da[q]), tv);
    }
  for (int p = 0; p < 4; ++p)
    for (int q = p + 1; q < 4; ++q)
      for (int r = 0; r < 4; ++r)
        for (int s = r + 1; s < 4; ++s) {
          double wv = I.w(dmode(p), dmode(q), dmode(r), dmode(s));
          if (wv != 0.0) HD = add(HD, mul(mul(Dc[p], Dc[q]), mul(Da[s], Da[r])), wv);
        }
  // S^D_p monomials: a_d (1/2 t_pd) and a+_q a_r a_s, s<r (<pq||sr>)
  struct Mono {
    Mat16 M;
    int q, s, r, d;  // d >= 0: single annihilator
  };
  std::vector<Mono> smono;
  for (int d = 0; d < 4; ++d) smono.push_back({Da[d], -1, -1, -1, d});
  for (int q = 0; q < 4; ++q)
    for (int s = 0; s < 4; ++s)
      for (int r = s + 1; r < 4; ++r) smono.push_back({mul(Dc[q], mul(Da[r], Da[s])), q, s, r, -1});
  auto smono_coef = [&](const Mono& m, int p) {
    if (m.d >= 0) return 0.5 * I.t(p, dmode(m.d));
    return I.w(p, dmode(m.q), dmode(m.s), dmode(m.r));
  };

  // ---- families
  auto F = [&](const Group* Lg, int Lbase, bool Lt, const Group* Rg, int Rbase, bool Rt, int count, const Mat16& D,
               int piD, int piR, double coef, const char* tag) {
    if (count <= 0 || zero(D) || coef == 0.0) return;
    if (Lg && (Lg->n() == 0 || Lg->lay.size == 0)) return;
    if (Rg && (Rg->n() == 0 || Rg->lay.size == 0)) return;
    SFam f;
    f.L = Lg;
    f.Lbase = Lbase;
    f.Lt = Lt;
    f.R = Rg;
    f.Rbase = Rbase;
    f.Rt = Rt;
    f.count = count;
    f.D = D;
    f.piD = piD;
    f.piR = piR;
    f.coef = coef;
    f.tag = tag;
    O.fams.push_back(f);
  };
  auto inter = [&](const Group& src, std::vector<std::vector<double>> rows) -> const Group* {
    bool nz = false;
    for (auto& r : rows)
      for (double x : r) nz |= (x != 0.0);
    if (!nz || src.n() == 0) return nullptr;
    std::vector<OpKey> nm(rows.size(), OpKey{'X', -1, -1});
    O.extra.push_back(bld.combine(src, rows, nm));
    return O.extra.back().get();
  };
  const Group* LG = L.g.data();
  const Group* RG = R.g.data();
  auto lcre = [&](int s) { return &LG[s ? G_CB : G_CA]; };
  auto rcre = [&](int s) { return &RG[s ? G_CB : G_CA]; };
  const int nLs[2] = {(int)Lca.size(), (int)Lcb.size()};
  const int nRs[2] = {R.g[G_CA].n(), R.g[G_CB].n()};

  // (4,0,0) (0,0,4) (0,4,0) and E_core
  F(&LG[G_H], 0, false, nullptr, 0, false, 1, Id, 0, 0, 1.0, "HL");
  F(nullptr, 0, false, &RG[G_H], 0, false, 1, Id, 0, 0, 1.0, "HR");
  F(nullptr, 0, false, nullptr, 0, false, 1, HD, 0, 0, 1.0, "HD");
  if (I.ecore != 0.0) F(nullptr, 0, false, nullptr, 0, false, 1, Id, 0, 0, I.ecore, "ecore");
  // (3,1,0): -S^L_d a+_d + S^L_d^T a_d ; S^L members are L's externals ascending (D modes first)
  for (int d = 0; d < 4; ++d) {
    const int gid = dspin(d) ? G_SB : G_SA;
    const int mem = d >> 1;  // C1 mode, then C2 mode of that spin
    F(&LG[gid], mem, false, nullptr, 0, false, 1, Dc[d], 1, 0, -1.0, "SLd");
    F(&LG[gid], mem, true, nullptr, 0, false, 1, Da[d], 1, 0, 1.0, "SLd+");
  }
  // (1,3,0): a+_p S^D_p - a_p S^D_p^T  -> per dot monomial an intermediate sum_p c(p) a+_p
  for (auto& m : smono)
    for (int s = 0; s < 2; ++s) {
      std::vector<double> c(nLs[s]);
      for (int i = 0; i < nLs[s]; ++i) c[i] = smono_coef(m, (*Lc[s])[i].p);
      const Group* Y = inter(*lcre(s), {c});
      if (!Y) continue;
      F(Y, 0, false, nullptr, 0, false, 1, m.M, 1, 0, 1.0, "pSD");
      F(Y, 0, true, nullptr, 0, false, 1, tr(m.M), 1, 0, -1.0, "pSD+");
    }
  // (3,0,1): -S^L_r a+_r + S^L_r^T a_r  (S^L members from index 2 are the R modes)
  for (int s = 0; s < 2; ++s) {
    const int gid = s ? G_SB : G_SA;
    F(&LG[gid], 2, false, rcre(s), 0, false, nRs[s], Id, 0, 1, -1.0, "SLr");
    F(&LG[gid], 2, true, rcre(s), 0, true, nRs[s], Id, 0, 1, 1.0, "SLr+");
  }
  // (1,0,3): a+_p S^R_p - a_p S^R_p^T (S^R members: L modes first)
  for (int s = 0; s < 2; ++s) {
    const int gid = s ? G_SB : G_SA;
    F(lcre(s), 0, false, &RG[gid], 0, false, nLs[s], Id, 0, 1, 1.0, "pSR");
    F(lcre(s), 0, true, &RG[gid], 0, true, nLs[s], Id, 0, 1, -1.0, "pSR+");
  }
  // (0,3,1): -S^D_r a+_r + S^D_r^T a_r  -> per dot monomial sum_r c(r) a+_r on R
  for (auto& m : smono)
    for (int s = 0; s < 2; ++s) {
      std::vector<double> c(nRs[s]);
      for (int i = 0; i < nRs[s]; ++i) c[i] = smono_coef(m, R.g[s ? G_CB : G_CA].names[i].p);
      const Group* Z = inter(*rcre(s), {c});
      if (!Z) continue;
      F(nullptr, 0, false, Z, 0, false, 1, m.M, 1, 1, -1.0, "SDr");
      F(nullptr, 0, false, Z, 0, true, 1, tr(m.M), 1, 1, 1.0, "SDr+");
    }
  // (0,1,3): a+_d S^R_d - a_d S^R_d^T  (S^R member of mode d is its orbital index)
  for (int d = 0; d < 4; ++d) {
    const int gid = dspin(d) ? G_SB : G_SA;
    const int mem = dmode(d) >> 1;
    F(nullptr, 0, false, &RG[gid], mem, false, 1, Dc[d], 1, 1, 1.0, "dSR");
    F(nullptr, 0, false, &RG[gid], mem, true, 1, Da[d], 1, 1, -1.0, "dSR+");
  }
  // (2,2,0): P^L_dd' A^D_dd' + h.c. + Q^L_dd' B^D_dd'
  for (int d = 0; d < 4; ++d)
    for (int e = 0; e < 4; ++e) {
      if (d < e) {
        const Group& src = LG[a_gid(dspin(d), dspin(e))];
        const Group* Y = inter(src, {coefW(src, dmode(d), dmode(e))});
        if (Y) {
          Mat16 AD = mul(Dc[d], Dc[e]);
          F(Y, 0, true, nullptr, 0, false, 1, AD, 0, 0, 1.0, "PLAD");
          F(Y, 0, false, nullptr, 0, false, 1, tr(AD), 0, 0, 1.0, "PLAD+");
        }
      }
      const Group& src = LG[q_src_gid(dspin(d), dspin(e))];
      const Group* Q = inter(src, {coefQ(src, dmode(d), dmode(e))});
      if (Q) F(Q, 0, false, nullptr, 0, false, 1, mul(Dc[d], Da[e]), 0, 0, 1.0, "QLBD");
    }
  // (0,2,2): A^D_dd' P^R_dd' + h.c. + B^D_dd' Q^R_dd'
  for (int d = 0; d < 4; ++d)
    for (int e = 0; e < 4; ++e) {
      if (d < e) {
        const Group* Y = YR[y_cls(dspin(d), dspin(e))];
        Mat16 AD = mul(Dc[d], Dc[e]);
        F(nullptr, 0, false, Y, ydd[d][e], true, 1, AD, 0, 0, 1.0, "ADPR");
        F(nullptr, 0, false, Y, ydd[d][e], false, 1, tr(AD), 0, 0, 1.0, "ADPR+");
      }
      F(nullptr, 0, false, QR[q_cls(dspin(d), dspin(e))], qdd[d][e], false, 1, mul(Dc[d], Da[e]), 0, 0, 1.0,
        "BDQR");
    }
  // (2,0,2): A^L_pq P^R_pq + h.c. + B^L_ps Q^R_ps  (member lists aligned)
  for (int c = 0; c < 3; ++c) {
    const int n = L.g[LAG[c]].n();
    F(&LG[LAG[c]], 0, false, YR[c], 0, true, n, Id, 0, 0, 1.0, "ALPR");
    F(&LG[LAG[c]], 0, true, YR[c], 0, false, n, Id, 0, 0, 1.0, "ALPR+");
    F(&LG[LQG[c]], 0, false, QR[c], 0, false, L.g[LQG[c]].n(), Id, 0, 0, 1.0, "BLQR");
  }
  // (2,1,1): P^L_dr a+_d a+_r - P^L_dr^T a_d a_r + Q^L_dr a+_d a_r - Q^L_rd a_d a+_r
  for (int d = 0; d < 4; ++d)
    for (int s = 0; s < 2; ++s) {
      const auto& rn = R.g[s ? G_CB : G_CA].names;
      if (rn.empty()) continue;
      std::vector<std::vector<double>> ry, rq1, rq2;
      const Group& sA = LG[a_gid(dspin(d), s)];
      const Group& sQ1 = LG[q_src_gid(dspin(d), s)];
      const Group& sQ2 = LG[q_src_gid(s, dspin(d))];
      for (auto& rk : rn) {
        ry.push_back(coefW(sA, dmode(d), rk.p));
        rq1.push_back(coefQ(sQ1, dmode(d), rk.p));
        rq2.push_back(coefQ(sQ2, rk.p, dmode(d)));
      }
      const int n = (int)rn.size();
      if (const Group* Y = inter(sA, ry)) {
        F(Y, 0, true, rcre(s), 0, false, n, Dc[d], 1, 1, 1.0, "PLdr");
        F(Y, 0, false, rcre(s), 0, true, n, Da[d], 1, 1, -1.0, "PLdr+");
      }
      if (const Group* Q1 = inter(sQ1, rq1)) F(Q1, 0, false, rcre(s), 0, true, n, Dc[d], 1, 1, 1.0, "QLdr");
      if (const Group* Q2 = inter(sQ2, rq2)) F(Q2, 0, false, rcre(s), 0, false, n, Da[d], 1, 1, -1.0, "QLrd");
    }
  // (1,1,2): a+_p a+_d P^R_pd - a_p a_d P^R_pd^T + a+_p a_d Q^R_pd - a_p a+_d Q^R_dp
  for (int d = 0; d < 4; ++d)
    for (int s = 0; s < 2; ++s) {
      const int n = nLs[s];
      const Group* Y = YR[y_cls(s, dspin(d))];
      F(lcre(s), 0, false, Y, yb[d][s], true, n, Dc[d], 1, 0, 1.0, "pdPR");
      F(lcre(s), 0, true, Y, yb[d][s], false, n, Da[d], 1, 0, -1.0, "pdPR+");
      F(lcre(s), 0, false, QR[q_cls(s, dspin(d))], qb1[d][s], false, n, Da[d], 1, 0, 1.0, "pdQR");
      F(lcre(s), 0, true, QR[q_cls(dspin(d), s)], qb2[d][s], false, n, Dc[d], 1, 0, -1.0, "dpQR");
    }
  // (1,2,1): -[sum_s a_s Q^D_rs + sum_q a+_q P^D_rq] a+_r + h.c.
  for (int s = 0; s < 2; ++s) {
    const auto& rn = R.g[s ? G_CB : G_CA].names;
    const int n = (int)rn.size();
    if (n == 0) continue;
    for (int q = 0; q < 4; ++q)
      for (int t = 0; t < 4; ++t) {
        // U_r = sum_{s' in L} <r q||s' t> a+_s'
        int ls = (dspin(q) == dspin(t)) ? s : (s == dspin(t) ? dspin(q) : -1);
        if (ls < 0) continue;
        std::vector<std::vector<double>> rows;
        for (auto& rk : rn) {
          std::vector<double> c(nLs[ls]);
          for (int i = 0; i < nLs[ls]; ++i) c[i] = I.w(rk.p, dmode(q), (*Lc[ls])[i].p, dmode(t));
          rows.push_back(c);
        }
        const Group* U = inter(*lcre(ls), rows);
        if (!U) continue;
        Mat16 M = mul(Dc[q], Da[t]);
        F(U, 0, true, rcre(s), 0, false, n, M, 0, 1, -1.0, "aQDr");
        F(U, 0, false, rcre(s), 0, true, n, tr(M), 0, 1, 1.0, "aQDr+");
      }
    for (int sd = 0; sd < 4; ++sd)
      for (int td = sd + 1; td < 4; ++td) {
        // V_r = sum_{q in L} <r q||s t> a+_q
        int qs;
        if (dspin(sd) == dspin(td))
          qs = (s == dspin(sd)) ? dspin(sd) : -1;
        else
          qs = (s == dspin(sd)) ? dspin(td) : dspin(sd);
        if (qs < 0) continue;
        std::vector<std::vector<double>> rows;
        for (auto& rk : rn) {
          std::vector<double> c(nLs[qs]);
          for (int i = 0; i < nLs[qs]; ++i) c[i] = I.w(rk.p, (*Lc[qs])[i].p, dmode(sd), dmode(td));
          rows.push_back(c);
        }
        const Group* V = inter(*lcre(qs), rows);
        if (!V) continue;
        Mat16 M = mul(Da[td], Da[sd]);
        F(V, 0, false, rcre(s), 0, false, n, M, 0, 1, -1.0, "cPDr");
        F(V, 0, true, rcre(s), 0, true, n, tr(M), 0, 1, 1.0, "cPDr+");
      }
  }
  for (auto& f : O.fams) O.nterms += f.count;
  dev_sync(stream);

  // ---- sigma plan
  auto eff = [](const Group* g, bool t, int ket, int* bra) -> int {
    const Layout& l = g->lay;
    if (!t) {
      int b = l.by_ket[ket];
      if (b >= 0) *bra = l.bra[b];
      return b;
    }
    int b = l.by_bra[ket];
    if (b >= 0) *bra = l.ket[b];
    return b;
  };
  struct RSrc {
    const Group* g;
    int base, count;
    bool t;
    std::vector<int> need;          // psi blocks needing X
    std::vector<int64_t> xoff;      // per psi block (or -1)
    int64_t stride = 0;
  };
  std::vector<RSrc> rs;
  std::map<std::tuple<const Group*, int, int, bool>, int> rs_id;
  std::vector<int> fam_rs(O.fams.size());
  const int nb = (int)O.blocks.size();
  // contribution enumeration: for family f and source block b, list (out block, D element)
  struct Hit {
    int out;
    double dv;
    int lb;          // stored L block or -1 (identity)
  };
  auto hits = [&](const SFam& f, const PsiBlk& b, std::vector<Hit>& out) {
    out.clear();
    int il2 = b.il, lb = -1;
    if (f.L) {
      lb = eff(f.L, f.Lt, b.il, &il2);
      if (lb < 0) return;
    }
    int ir2 = b.ir;
    if (f.R) {
      if (eff(f.R, f.Rt, b.ir, &ir2) < 0) return;
    }
    for (int e2 = 0; e2 < 16; ++e2) {
      double dv = f.D[e2 * 16 + b.e];
      if (dv == 0.0) continue;
      int ob = O.find_block(il2, e2, ir2);
      if (ob < 0) continue;
      out.push_back({ob, dv, lb});
    }
  };
  std::vector<Hit> hv;
  for (size_t fi = 0; fi < O.fams.size(); ++fi) {
    const SFam& f = O.fams[fi];
    if (!f.R) {
      fam_rs[fi] = -1;
      continue;
    }
    auto key = std::make_tuple(f.R, f.Rbase, f.count, f.Rt);
    auto it = rs_id.find(key);
    int id;
    if (it == rs_id.end()) {
      id = (int)rs.size();
      rs_id[key] = id;
      RSrc r;
      r.g = f.R;
      r.base = f.Rbase;
      r.count = f.count;
      r.t = f.Rt;
      r.xoff.assign(nb, -1);
      rs.push_back(std::move(r));
    } else {
      id = it->second;
    }
    fam_rs[fi] = id;
    RSrc& r = rs[id];
    for (int bi = 0; bi < nb; ++bi) {
      hits(f, O.blocks[bi], hv);
      if (!hv.empty() && r.xoff[bi] < 0) r.xoff[bi] = 0;
    }
  }
  // psi blocks grouped by right sector (then block order): the R-step reads
  // psi from this permuted copy, so that the blocks one R operator block
  // multiplies stack into one tall operand (Eq. sigmablk56 for all of them at
  // once: same K and the same right factor), with far fewer partial tiles
  O.permbuf = tab.add(nullptr);
  std::vector<int> perm(nb);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return O.blocks[a].ir < O.blocks[b].ir; });
  std::vector<int> perm_pos(nb);
  O.perm_off.assign(nb, 0);
  {
    int64_t off = 0;
    for (int i = 0; i < nb; ++i) {
      perm_pos[perm[i]] = i;
      O.perm_off[perm[i]] = off;
      off += (int64_t)O.blocks[perm[i]].dl * O.blocks[perm[i]].dr;
    }
  }
  for (auto& r : rs) {
    // X blocks in the permuted order too, so that a run of stacked psi blocks
    // writes one stacked X (rows of the run, leading dimension d_R')
    for (int i = 0; i < nb; ++i) {
      const int bi = perm[i];
      if (r.xoff[bi] < 0) continue;
      int ir2 = -1;
      eff(r.g, r.t, O.blocks[bi].ir, &ir2);
      r.xoff[bi] = r.stride;
      r.need.push_back(bi);
      r.stride += (int64_t)O.blocks[bi].dl * O.Rb.dim[ir2];
    }
  }
  // pieces: (rsrc, t0, t1) packed into chunks of at most x_budget bytes
  struct Piece {
    int src, t0, t1;
    int64_t xbase;
  };
  std::vector<std::vector<Piece>> chunk_pieces;
  {
    const int64_t budget = (int64_t)(opt.x_budget / sizeof(double));
    std::vector<Piece> cur;
    int64_t used = 0, maxused = 0;
    for (int id = 0; id < (int)rs.size(); ++id) {
      const RSrc& r = rs[id];
      if (r.stride == 0) continue;
      int t = 0;
      while (t < r.count) {
        int64_t room = budget - used;
        int fit = (int)std::min<int64_t>(r.count - t, room / r.stride);
        if (fit <= 0) {
          if (cur.empty()) {
            fit = 1;  // a single member larger than the budget
          } else {
            chunk_pieces.push_back(cur);
            cur.clear();
            used = 0;
            continue;
          }
        }
        cur.push_back({id, t, t + fit, used});
        used += r.stride * fit;
        maxused = std::max(maxused, used);
        t += fit;
      }
    }
    if (!cur.empty()) chunk_pieces.push_back(cur);
    // two scratch slots: the R-step of chunk i writes slot i%2 while the
    // L-step of chunk i-1 (same launch) reads the other one
    O.Xbytes = (size_t)std::max<int64_t>(1, maxused) * sizeof(double);
    for (int sl = 0; sl < 2; ++sl) {
      O.X[sl] = (double*)dev_alloc(chunk_pieces.size() > (size_t)sl ? O.Xbytes : 256);
      O.Xbuf[sl] = tab.add(O.X[sl]);
    }
  }
  const int nrchunks = (int)chunk_pieces.size();
  // identity-R families form an extra chunk without an R-step
  chunk_pieces.push_back({{-1, 0, 0, 0}});
  O.pbuf = tab.add(nullptr);  // split-k partials (allocated once the plan is sized)
  int64_t partial_max = 0;    // doubles

  std::vector<GemmList> Rl(chunk_pieces.size()), Ll(chunk_pieces.size());
  for (size_t ci = 0; ci < chunk_pieces.size(); ++ci) {
    GemmList& rstep = Rl[ci];
    GemmList& lstep = Ll[ci];
    const int xb = (int)ci < nrchunks ? O.Xbuf[ci % 2] : -1;
    const auto& pcs = chunk_pieces[ci];
    // R-step
    for (const Piece& pc : pcs) {
      if (pc.src < 0) continue;
      const RSrc& r = rs[pc.src];
      const Layout& rl = r.g->lay;
      // runs of needed blocks that are neighbours in the permuted psi (same
      // right sector): one task each, its rows the blocks' rows stacked
      for (size_t j0 = 0; j0 < r.need.size();) {
        const PsiBlk& b = O.blocks[r.need[j0]];
        size_t j1 = j0 + 1;
        int rows = b.dl;
        while (j1 < r.need.size() && O.blocks[r.need[j1]].ir == b.ir &&
               perm_pos[r.need[j1]] == perm_pos[r.need[j1 - 1]] + 1) {
          rows += O.blocks[r.need[j1]].dl;
          ++j1;
        }
        int ir2 = -1;
        int sb = eff(r.g, r.t, b.ir, &ir2);
        const int dr2 = O.Rb.dim[ir2];
        rstep.begin(rows, dr2, pc.t1 - pc.t0, xb, pc.xbase + r.xoff[r.need[j0]], dr2, r.stride, false);
        GContrib c = make_contrib(b.dr, r.t ? 0 : GF_TRANS_B, O.permbuf, O.perm_off[r.need[j0]], b.dr, r.g->buf,
                                  (int64_t)(r.base + pc.t0) * r.g->stride() + rl.off[sb], r.t ? dr2 : b.dr, 1.0);
        c.b_bstride = r.g->stride();
        rstep.add(c);
        rstep.end();
        j0 = j1;
      }
    }
    // L-step: contributions grouped by output block
    std::vector<std::vector<GContrib>> per_out(nb);
    for (const Piece& pc : pcs) {
      for (size_t fi = 0; fi < O.fams.size(); ++fi) {
        const SFam& f = O.fams[fi];
        if (fam_rs[fi] != pc.src) continue;
        int t0 = pc.t0, t1 = pc.t1;
        if (pc.src < 0) {
          t0 = 0;
          t1 = f.count;
        }
        const RSrc* r = pc.src >= 0 ? &rs[pc.src] : nullptr;
        for (int bi = 0; bi < nb; ++bi) {
          const PsiBlk& b = O.blocks[bi];
          hits(f, b, hv);
          if (hv.empty()) continue;
          int zeta_par = f.piD * O.Lb.qn[b.il].n() + f.piR * (O.Lb.qn[b.il].n() + dot::nelec(b.e));
          double zeta = (zeta_par & 1) ? -1.0 : 1.0;
          for (const Hit& h : hv) {
            const PsiBlk& ob = O.blocks[h.out];
            GContrib c{};
            c.K = b.dl;
            c.nred = t1 - t0;
            c.alpha = f.coef * h.dv * zeta;
            c.s_buf = -1;
            if (f.L) {
              const Layout& ll = f.L->lay;
              c.a_buf = f.L->buf;
              c.a_off = (int64_t)(f.Lbase + t0) * f.L->stride() + ll.off[h.lb];
              c.lda = f.Lt ? ob.dl : b.dl;
              c.flags = f.Lt ? GF_TRANS_A : 0;
              c.a_rstride = f.L->stride();
            } else {
              c.flags = GF_IDENT_A;
              c.a_buf = 0;
            }
            if (r) {
              c.b_buf = xb;
              c.b_off = pc.xbase + r->xoff[bi];
              c.ldb = ob.dr;
              c.b_rstride = r->stride;
            } else {
              c.b_buf = 0;
              c.b_off = b.off;
              c.ldb = b.dr;
              c.b_rstride = 0;
            }
            per_out[h.out].push_back(c);
          }
        }
      }
    }
    // One task per output block.  A task whose k loop (contributions x
    // members x k tiles) is longer than opt.ksplit_tiles is cut at member
    // boundaries into parts of about equal length: the first part adds into
    // sigma, the others write partial blocks that the launch's reduction then
    // adds into sigma one after the other.  Every launch shape sees the same
    // parts, so results stay the same across shapes.
    int64_t pused = 0;
    for (int bo = 0; bo < nb; ++bo) {
      if (per_out[bo].empty()) continue;
      const PsiBlk& ob = O.blocks[bo];
      int64_t kt = 0;
      for (const GContrib& c : per_out[bo])
        if (!(c.flags & GF_IDENT_A)) kt += (int64_t)c.nred * ((c.K + 31) / 32);
      const int64_t nparts = std::max<int64_t>(1, (kt + opt.ksplit_tiles - 1) / opt.ksplit_tiles);
      lstep.begin(ob.dl, ob.dr, 1, 1, ob.off, ob.dr, 0, true);
      for (const GContrib& c : per_out[bo])
        if (c.flags & GF_IDENT_A) lstep.add(c);
      const int64_t target = (kt + nparts - 1) / nparts, blk = (int64_t)ob.dl * ob.dr;
      int64_t in_part = 0, part = 0;
      for (const GContrib& c : per_out[bo]) {
        if (c.flags & GF_IDENT_A) continue;
        const int64_t per = (c.K + 31) / 32;
        for (int m = 0; m < c.nred;) {
          if (in_part >= target && part + 1 < nparts) {
            lstep.end();
            lstep.begin(ob.dl, ob.dr, 1, O.pbuf, pused + part * blk, ob.dr, 0, false);
            lstep.tasks.back().accumulate |= GT_C64;
            ++part;
            in_part = 0;
          }
          // the last part takes every member left in one piece
          const int take = part + 1 >= nparts
                               ? c.nred - m
                               : (int)std::max<int64_t>(
                                     1, std::min<int64_t>(c.nred - m, (target - in_part + per - 1) / per));
          GContrib d = c;
          d.nred = take;
          d.a_off += (int64_t)m * c.a_rstride;
          d.b_off += (int64_t)m * c.b_rstride;
          d.s_off += (int64_t)m * c.s_rstride;
          lstep.add(d);
          in_part += take * per;
          m += take;
        }
      }
      lstep.end();
      if (part > 0) {
        ReduceSeg r{};
        r.dst_buf = 1;
        r.src_buf = O.pbuf;
        r.nsrc = (int32_t)part;
        r.dst_off = ob.off;
        r.src_off = pused;
        r.src_stride = blk;
        r.n = blk;
        lstep.reduce.push_back(r);
        pused += part * blk;
      }
    }
    partial_max = std::max(partial_max, pused);
    O.flops_r += rstep.flops;
    O.flops_l += lstep.flops;
    O.ngemm_r += rstep.ngemm;
    O.ngemm_l += lstep.ngemm;
  }
  {
    std::vector<int64_t> seg;
    for (int bi = 0; bi < nb; ++bi) {
      const int64_t n = (int64_t)O.blocks[bi].dl * O.blocks[bi].dr;
      if (n == 0) continue;
      seg.push_back(O.blocks[bi].off);
      seg.push_back(O.perm_off[bi]);
      seg.push_back(n);
    }
    O.nperm_seg = (int)(seg.size() / 3);
    O.perm_seg = (int64_t*)dev_alloc(sizeof(int64_t) * std::max<size_t>(3, seg.size()));
    if (!seg.empty()) dev_h2d(O.perm_seg, seg.data(), sizeof(int64_t) * seg.size());
    O.psi_perm = (double*)dev_alloc(sizeof(double) * (size_t)std::max<int64_t>(1, O.npsi));
    tab.set(O.permbuf, O.psi_perm);
  }
  O.partial_bytes = (size_t)std::max<int64_t>(1, partial_max) * sizeof(double);
  O.partial = (double*)dev_alloc(partial_max > 0 ? O.partial_bytes : 256);
  tab.set(O.pbuf, O.partial);
  // launches: [L(identity) + R(0)], [L(0) + R(1)], ..., [L(n-2) + R(n-1)], [L(n-1)];
  // the L-step of one chunk shares a launch with the R-step of the next one
  // so that the short R-step jobs fill the tail of the long L-step jobs.
  {
    const int n = nrchunks;
    GemmList& Lid = Ll[n];
    std::set<int> bufs;
    for (int i = 0; i <= n; ++i) {
      std::vector<GemmList*> parts;
      if (i == 0)
        parts.push_back(&Lid);
      else
        parts.push_back(&Ll[i - 1]);
      if (i < n) parts.push_back(&Rl[i]);
      GemmList m = GemmList::merge_by_cost(parts);
      if (m.tasks.empty()) continue;
      for (const GTask& t : m.tasks) bufs.insert(t.c_buf);
      for (const ReduceSeg& r : m.reduce) {
        bufs.insert(r.dst_buf);
        bufs.insert(r.src_buf);
      }
      for (const GContrib& c : m.contribs) {
        if (!(c.flags & GF_IDENT_A)) bufs.insert(c.a_buf);
        bufs.insert(c.b_buf);
        if (c.s_buf >= 0) bufs.insert(c.s_buf);
        DMRG_CHECK(c.b_buf != 1 && ((c.flags & GF_IDENT_A) || c.a_buf != 1), DMRG_EINTERNAL,
                   "sigma plan reads its output buffer");
      }
      m.upload(TILE_64x64);
      O.launches.push_back(std::move(m));
    }
    O.sigma_bufs.assign(bufs.begin(), bufs.end());
  }
  // operator memory kept for sigma
  auto gbytes = [](const Group& g) { return g.dev ? 8.0 * g.n() * (double)g.lay.size : 0.0; };
  for (auto& g : O.L->g) O.op_bytes += gbytes(g);
  for (auto& g : O.R->g) O.op_bytes += gbytes(g);
  for (auto& g : O.extra) O.op_bytes += gbytes(*g);
  O.build_flops = bld.st.flops;
  dev_sync(stream);
  O.build_seconds = wall_seconds() - t0;
  return ops;
}

// ----------------------------------------------------------------------------
void gather_psi(Ops& O, const double* psi, int prec, void* stream) {
  k_copy_segments(psi, O.psi_perm, O.perm_seg, O.nperm_seg, stream);
  if (prec != P_F64) k_d2f(O.psi_perm, O.psi_perm32, O.npsi, stream);
}

void sigma_run(Ops& O, const double* psi, double* sigma, int prec, void* stream) {
  DMRG_CHECK(prec == P_F64 || prec == P_F32 || prec == P_BF16X3, DMRG_EINVAL, "unknown precision");
  DevTable* tab = O.tab.get();
  const void* p0 = psi;
  if (prec != P_F64) {
    make_reduced_copies(O, stream);
    k_d2f(psi, O.psi32, O.npsi, stream);
    tab = O.tab32.get();
    p0 = O.psi32;
  }
  const bool tuned = O.tile_choice[prec].size() == O.launches.size();
  auto launch = [&](size_t i) {
    GemmList& l = O.launches[i];
    l.grid_per_xcd = tuned ? O.grid_choice[prec][i] : 0;
    l.run_tile(tuned ? O.tile_choice[prec][i] : TILE_64x64, *tab, p0, sigma, prec, stream);
  };
  k_fill(sigma, 0.0, O.npsi, stream);
  gather_psi(O, psi, prec, stream);
  if (!O.profile) {
    for (size_t i = 0; i < O.launches.size(); ++i) launch(i);
    return;
  }
  while (O.events.size() < O.launches.size() + 1) O.events.push_back(ev_create());
  ev_record(O.events[0], stream);
  for (size_t i = 0; i < O.launches.size(); ++i) {
    launch(i);
    ev_record(O.events[i + 1], stream);
  }
  for (size_t i = 0; i < O.launches.size(); ++i) O.prof_ms += ev_elapsed_ms(O.events[i], O.events[i + 1]);
  O.prof_launches += (int64_t)O.launches.size();
  ++O.prof_calls;
}

void autotune_launches(size_t nl, const std::function<void(const std::vector<int>&, const std::vector<int64_t>&,
                                                           std::vector<double>&)>& run_all,
                       std::vector<int>& tiles, std::vector<int64_t>& grids, double& ms_default, double& ms_best) {
  std::vector<double> ms(nl), best(nl, 1e300), ms_default_i(nl, 0.0);
  tiles.assign(nl, TILE_64x64);
  grids.assign(nl, 0);
  std::vector<int> tv(nl);
  std::vector<int64_t> gv(nl, 0);
  ms_default = 0;
  for (int t = 0; t < NTILE; ++t) {
    std::fill(tv.begin(), tv.end(), t);
    // one workgroup per job (the first run also uploads this shape's lists),
    // then resident workgroups taking cost-balanced units (grid -1)
    for (int64_t g : {int64_t(0), int64_t(0), int64_t(-1)}) {
      std::fill(gv.begin(), gv.end(), g);
      run_all(tv, gv, ms);
      for (size_t i = 0; i < nl; ++i) {
        if (t == TILE_64x64 && g == 0) ms_default_i[i] = ms[i];
        if (ms[i] < best[i]) {
          best[i] = ms[i];
          tiles[i] = t;
          grids[i] = g;
        }
      }
    }
  }
  ms_default = 0;
  ms_best = 0;
  for (size_t i = 0; i < nl; ++i) {
    ms_default += ms_default_i[i];
    ms_best += best[i];
  }
}

void sigma_autotune(Ops& O, int prec, void* stream) {
  DMRG_CHECK(prec == P_F64 || prec == P_F32 || prec == P_BF16X3, DMRG_EINVAL, "unknown precision");
  const size_t nl = O.launches.size();
  double* psi = (double*)dev_alloc(sizeof(double) * (size_t)O.npsi);
  double* sig = (double*)dev_alloc(sizeof(double) * (size_t)O.npsi);
  k_fill(psi, 1.0 / std::sqrt((double)O.npsi), O.npsi, stream);
  DevTable* tab = O.tab.get();
  const void* p0 = psi;
  if (prec != P_F64) {
    make_reduced_copies(O, stream);
    k_d2f(psi, O.psi32, O.npsi, stream);
    tab = O.tab32.get();
    p0 = O.psi32;
  }
  gather_psi(O, psi, prec, stream);
  while (O.events.size() < nl + 1) O.events.push_back(ev_create());
  auto run_all = [&](const std::vector<int>& tiles, const std::vector<int64_t>& grids, std::vector<double>& ms) {
    k_fill(sig, 0.0, O.npsi, stream);
    ev_record(O.events[0], stream);
    for (size_t i = 0; i < nl; ++i) {
      O.launches[i].grid_per_xcd = grids[i];
      O.launches[i].run_tile(tiles[i], *tab, p0, sig, prec, stream);
      ev_record(O.events[i + 1], stream);
    }
    for (size_t i = 0; i < nl; ++i) ms[i] = ev_elapsed_ms(O.events[i], O.events[i + 1]);
  };
  try {
    autotune_launches(nl, run_all, O.tile_choice[prec], O.grid_choice[prec], O.tune_ms_default[prec],
                      O.tune_ms_best[prec]);
  } catch (...) {
    dev_free(psi);
    dev_free(sig);
    throw;
  }
  dev_sync(stream);
  dev_free(psi);
  dev_free(sig);
  // keep the device task lists of the shapes in use (64x64 serves untuned precisions)
  for (size_t i = 0; i < nl; ++i) {
    bool keep[NTILE] = {true};
    for (int q = 0; q < 3; ++q)
      if (O.tile_choice[q].size() == nl) keep[O.tile_choice[q][i]] = true;
    for (int t = 0; t < NTILE; ++t)
      if (!keep[t]) O.launches[i].release_tile(t);
  }
}

// diag(H): families whose effective left and right operators conserve the
// block quantum numbers contribute  c D_ee zeta sum_t diag(L_t)_l diag(R_t)_r.
void diag_run(Ops& O, double* diag, void* stream) {
  DevTable& tab = *O.tab;
  k_fill(diag, 0.0, O.npsi, stream);
  const int64_t nL = O.Lb.total, nR = O.Rb.total;
  auto diag_meta = [](const Group& g, const Basis& B, std::vector<int64_t>& meta) {
    meta.clear();
    for (int bk = 0; bk < g.lay.nblk(); ++bk) {
      if (g.lay.bra[bk] != g.lay.ket[bk]) continue;
      int s = g.lay.ket[bk];
      meta.push_back(g.lay.off[bk]);
      meta.push_back(B.dim[s]);
      meta.push_back(B.off[s]);
    }
  };
  std::vector<int64_t> meta;
  for (const SFam& f : O.fams) {
    bool dz = true;
    if (f.L && !(f.L->dq == QN(0, 0))) dz = false;
    if (f.R && !(f.R->dq == QN(0, 0))) dz = false;
    if (!dz) continue;
    bool anyd = false;
    for (int e = 0; e < 16; ++e) anyd |= f.D[e * 16 + e] != 0.0;
    if (!anyd) continue;
    const int cnt = f.count;
    double* dL = (double*)dev_alloc(sizeof(double) * (size_t)cnt * nL);
    double* dR = (double*)dev_alloc(sizeof(double) * (size_t)cnt * nR);
    int64_t* dmeta = nullptr;
    if (f.L) {
      diag_meta(*f.L, O.Lb, meta);
      dmeta = (int64_t*)dev_alloc(sizeof(int64_t) * std::max<size_t>(1, meta.size()));
      dev_h2d(dmeta, meta.data(), meta.size() * sizeof(int64_t));
      k_gather_diag(f.L->dev + (int64_t)f.Lbase * f.L->stride(), dmeta, (int)meta.size() / 3, f.L->stride(), nL,
                    cnt, dL, stream);
      dev_sync(stream);
      dev_free(dmeta);
    } else {
      k_fill(dL, 1.0, (int64_t)cnt * nL, stream);
    }
    if (f.R) {
      diag_meta(*f.R, O.Rb, meta);
      dmeta = (int64_t*)dev_alloc(sizeof(int64_t) * std::max<size_t>(1, meta.size()));
      dev_h2d(dmeta, meta.data(), meta.size() * sizeof(int64_t));
      k_gather_diag(f.R->dev + (int64_t)f.Rbase * f.R->stride(), dmeta, (int)meta.size() / 3, f.R->stride(), nR,
                    cnt, dR, stream);
      dev_sync(stream);
      dev_free(dmeta);
    } else {
      k_fill(dR, 1.0, (int64_t)cnt * nR, stream);
    }
    int bl = tab.add(dL), br = tab.add(dR);
    GemmList gl;
    for (const PsiBlk& b : O.blocks) {
      double dv = f.D[b.e * 16 + b.e];
      if (dv == 0.0) continue;
      int zp = f.piD * O.Lb.qn[b.il].n() + f.piR * (O.Lb.qn[b.il].n() + dot::nelec(b.e));
      double zeta = (zp & 1) ? -1.0 : 1.0;
      gl.begin(b.dl, b.dr, 1, 1, b.off, b.dr, 0, true);
      gl.add(make_contrib(cnt, GF_TRANS_A, bl, O.Lb.off[b.il], (int)nL, br, O.Rb.off[b.ir], (int)nR,
                          f.coef * dv * zeta));
      gl.end();
    }
    gl.upload();
    gl.run(tab, nullptr, diag, P_F64, stream);
    dev_sync(stream);
    tab.set(bl, nullptr);
    tab.set(br, nullptr);
    dev_free(dL);
    dev_free(dR);
  }
  dev_sync(stream);  // also when no family contributes (the fill above)
}

// The same sum as diag_run, for callers that cannot allocate: the members of
// a family are taken in chunks whose diagonals fit the scratch next to the
// chunk's task list, and each chunk adds its part to diag (binary64).  A
// family that fits in one chunk gives bit-identical results; with several
// chunks the partial sums are rounded once more per chunk.
void diag_run_noalloc(Ops& O, double* diag, void* stream, void* scratch, size_t cap) {
  constexpr size_t TASKLIST_RESERVE = size_t(4) << 20;  // task list, buckets, units of one chunk
  k_fill(diag, 0.0, O.npsi, stream);
  const int64_t nL = O.Lb.total, nR = O.Rb.total;
  auto diag_meta = [](const Group& g, const Basis& B, std::vector<int64_t>& meta) {
    meta.clear();
    for (int bk = 0; bk < g.lay.nblk(); ++bk) {
      if (g.lay.bra[bk] != g.lay.ket[bk]) continue;
      int s = g.lay.ket[bk];
      meta.push_back(g.lay.off[bk]);
      meta.push_back(B.dim[s]);
      meta.push_back(B.off[s]);
    }
  };
  Arena A;
  A.base = (char*)scratch;
  A.cap = cap;
  std::vector<int64_t> metaL, metaR;
  for (const SFam& f : O.fams) {
    bool dz = true;
    if (f.L && !(f.L->dq == QN(0, 0))) dz = false;
    if (f.R && !(f.R->dq == QN(0, 0))) dz = false;
    if (!dz) continue;
    bool anyd = false;
    for (int e = 0; e < 16; ++e) anyd |= f.D[e * 16 + e] != 0.0;
    if (!anyd) continue;
    if (f.L) diag_meta(*f.L, O.Lb, metaL);
    if (f.R) diag_meta(*f.R, O.Rb, metaR);
    const size_t fixed = 4 * sizeof(void*) + (metaL.size() + metaR.size()) * sizeof(int64_t) + 4 * 256 +
                         TASKLIST_RESERVE;
    const size_t per_member = (size_t)(nL + nR) * sizeof(double);
    DMRG_CHECK(cap > fixed + per_member + 512, DMRG_ENOMEM,
               "diag without allocation: one member's diagonals (" + std::to_string(per_member) +
                   " bytes) and a chunk's task list do not fit the " + std::to_string(cap) + "-byte static scratch");
    int64_t chunk = (int64_t)((cap - fixed - 512) / per_member);
    if (chunk >= 32) chunk -= chunk % 32;  // whole k tiles per chunk
    for (int64_t t0 = 0; t0 < f.count; t0 += chunk) {
      const int c = (int)std::min<int64_t>(chunk, f.count - t0);
      dev_sync(stream);  // the previous chunk's kernels no longer read the scratch
      A.reset();
      void** dtab = (void**)A.take(4 * sizeof(void*));
      double* dL = (double*)A.take(sizeof(double) * (size_t)c * nL);
      double* dR = (double*)A.take(sizeof(double) * (size_t)c * nR);
      void* tab_h[4] = {nullptr, nullptr, dL, dR};
      dev_h2d(dtab, tab_h, sizeof tab_h);
      if (f.L) {
        int64_t* dm = (int64_t*)A.take(sizeof(int64_t) * std::max<size_t>(1, metaL.size()));
        dev_h2d(dm, metaL.data(), metaL.size() * sizeof(int64_t));
        k_gather_diag(f.L->dev + (int64_t)(f.Lbase + t0) * f.L->stride(), dm, (int)metaL.size() / 3,
                      f.L->stride(), nL, c, dL, stream);
      } else {
        k_fill(dL, 1.0, (int64_t)c * nL, stream);
      }
      if (f.R) {
        int64_t* dm = (int64_t*)A.take(sizeof(int64_t) * std::max<size_t>(1, metaR.size()));
        dev_h2d(dm, metaR.data(), metaR.size() * sizeof(int64_t));
        k_gather_diag(f.R->dev + (int64_t)(f.Rbase + t0) * f.R->stride(), dm, (int)metaR.size() / 3,
                      f.R->stride(), nR, c, dR, stream);
      } else {
        k_fill(dR, 1.0, (int64_t)c * nR, stream);
      }
      GemmList gl;
      for (const PsiBlk& b : O.blocks) {
        double dv = f.D[b.e * 16 + b.e];
        if (dv == 0.0) continue;
        int zp = f.piD * O.Lb.qn[b.il].n() + f.piR * (O.Lb.qn[b.il].n() + dot::nelec(b.e));
        double zeta = (zp & 1) ? -1.0 : 1.0;
        gl.begin(b.dl, b.dr, 1, 1, b.off, b.dr, 0, true);
        gl.add(make_contrib(c, GF_TRANS_A, 2, O.Lb.off[b.il], (int)nL, 3, O.Rb.off[b.ir], (int)nR,
                            f.coef * dv * zeta));
        gl.end();
      }
      gl.upload(TILE_64x64, &A);
      gl.run_uploaded(TILE_64x64, dtab, nullptr, diag, P_F64, stream);
    }
  }
  dev_sync(stream);
}

void make_reduced_copies(Ops& O, void* stream) {
  if (O.tab32) return;
  auto t32 = std::make_unique<DevTable>();
  while (t32->size() < O.tab->size()) t32->add(nullptr);
  std::set<int> need(O.sigma_bufs.begin(), O.sigma_bufs.end());
  need.erase(0);
  need.erase(1);
  auto convert = [&](Group& g) {
    if (!g.dev || !need.count(g.buf)) return;
    const int64_t n = (int64_t)g.n() * g.lay.size;
    if (!g.dev32) {
      g.dev32 = (float*)dev_alloc(sizeof(float) * (size_t)std::max<int64_t>(1, n));
      k_d2f(g.dev, g.dev32, n, stream);
    }
    t32->set(g.buf, g.dev32);
    O.op_bytes32 += 4.0 * (double)n;
    need.erase(g.buf);
  };
  for (auto& g : O.L->g) convert(g);
  for (auto& g : O.R->g) convert(g);
  for (auto& g : O.extra) convert(*g);
  for (int sl = 0; sl < 2; ++sl) {
    if (!need.count(O.Xbuf[sl])) continue;
    O.X32[sl] = (float*)dev_alloc(std::max<size_t>(256, O.Xbytes / 2));
    t32->set(O.Xbuf[sl], O.X32[sl]);
    need.erase(O.Xbuf[sl]);
  }
  if (need.count(O.permbuf)) {
    O.psi_perm32 = (float*)dev_alloc(sizeof(float) * (size_t)std::max<int64_t>(1, O.npsi));
    t32->set(O.permbuf, O.psi_perm32);
    need.erase(O.permbuf);
  }
  if (need.count(O.pbuf)) {  // split-k partials are binary64 in every precision
    t32->set(O.pbuf, O.partial);
    need.erase(O.pbuf);
  }
  DMRG_CHECK(need.empty(), DMRG_EINTERNAL, "sigma plan reads a buffer without a reduced-precision copy");
  O.psi32 = (float*)dev_alloc(sizeof(float) * (size_t)O.npsi);
  dev_sync(stream);
  O.tab32 = std::move(t32);
}


}  // namespace dmrg
