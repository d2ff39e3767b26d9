// Decimation of the two-dot wavefunction (the truncation step of the two-dot
// sweep, paper Sec. 2.1: after the two-dot problem is solved, the enlarged
// block's new renormalized states are the D most important states of the
// two-dot vector, and the weight of the states dropped is the discarded
// weight).
//
// The vector is split at the bond between the dots.  For every symmetry
// sector q of that bond (electron numbers of the sites to its left), the
// reduced density matrix of one side,
//   direction 0 (left):  rho_q = sum over right parts (n2, r) of M_q M_q^T,
//                        rows (l, n1) with q(l) + q(n1) = q,
//   direction 1 (right): rows (n2, r) with q(r) - q(n2) = q,
// is formed on the GPU from the psi blocks (grouped GEMM kernel) and
// diagonalised (rocSOLVER).  Its eigenvalues are the squared Schmidt
// coefficients.  The D largest over all sectors are kept (with cutoff > 0
// only those above cutoff <psi|psi>; with cutoff 0 zero weights as well, so
// that a large D keeps the enlarged block's whole space); their eigenvectors become the new site tensor: left-canonical
// A[k] (direction 0) or right-canonical A[k+1] (direction 1), whose
// columns (rows) are orthonormal because the eigenvectors are.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>

#include "ops.h"

namespace dmrg {

void decimate_run(Ops& O, const double* psi, int D, int direction, double cutoff, void* stream) {
  DMRG_CHECK(D > 0, DMRG_EINVAL, "bond dimension must be positive");
  DMRG_CHECK(direction == 0 || direction == 1, DMRG_EINVAL, "direction must be 0 (left) or 1 (right)");
  DMRG_CHECK(cutoff >= 0 && cutoff < 1, DMRG_EINVAL, "cutoff must lie in [0, 1)");
  // row blocks (the kept side) and column blocks (the traced side) of every sector
  struct RowBlk {
    int a0, a1;   // (il, n1) for direction 0, (n2, ir) for direction 1
    int dim;
    int off = 0;  // row offset inside rho_q
  };
  std::map<QN, std::vector<RowBlk>> rows;  // sorted by (q_alpha, q_beta)
  auto key_of = [&](const PsiBlk& b, int* a0, int* a1, int* dim) {
    const int n1 = b.e / 4, n2 = b.e % 4;
    if (direction == 0) {
      *a0 = b.il;
      *a1 = n1;
      *dim = b.dl;
      return O.Llabel[b.il] + SITE_QN[n1];
    }
    *a0 = n2;
    *a1 = b.ir;
    *dim = b.dr;
    return O.Rlabel[b.ir] - SITE_QN[n2];
  };
  for (const PsiBlk& b : O.blocks) {
    int a0, a1, dim;
    const QN q = key_of(b, &a0, &a1, &dim);
    auto& v = rows[q];
    bool have = false;
    for (auto& r : v) have |= r.a0 == a0 && r.a1 == a1;
    if (!have) v.push_back({a0, a1, dim});
  }
  struct Sec {
    QN q;
    int n = 0;
    int64_t rho_off = 0, w_off = 0;
  };
  std::vector<Sec> secs;
  int64_t rho_total = 0, w_total = 0;
  int nmax = 0;
  for (auto& kv : rows) {
    auto& v = kv.second;
    std::sort(v.begin(), v.end(), [](const RowBlk& x, const RowBlk& y) {
      return x.a0 != y.a0 ? x.a0 < y.a0 : x.a1 < y.a1;
    });
    Sec s;
    s.q = kv.first;
    for (auto& r : v) {
      r.off = s.n;
      s.n += r.dim;
    }
    s.rho_off = rho_total;
    s.w_off = w_total;
    rho_total += (int64_t)s.n * s.n;
    w_total += s.n;
    nmax = std::max(nmax, s.n);
    secs.push_back(s);
  }
  auto row_index = [&](const QN& q, int a0, int a1) -> const RowBlk* {
    for (const auto& r : rows[q])
      if (r.a0 == a0 && r.a1 == a1) return &r;
    return nullptr;
  };
  std::map<QN, int> sec_index;
  for (int i = 0; i < (int)secs.size(); ++i) sec_index[secs[i].q] = i;

  // rho_q[a][b] = sum_c psi(a, c) op psi(b, c): one task per pair of row
  // blocks, one contribution per psi block pair sharing the traced part c
  double* rho = (double*)dev_alloc(sizeof(double) * (size_t)std::max<int64_t>(1, rho_total));
  double* w = (double*)dev_alloc(sizeof(double) * (size_t)std::max<int64_t>(1, w_total));
  double* work = (double*)dev_alloc(sizeof(double) * (size_t)std::max(1, nmax));
  int* info = (int*)dev_alloc(sizeof(int) * std::max<size_t>(1, secs.size()));
  DevTable tab;
  const int rbuf = tab.add(rho);
  struct Entry {
    const PsiBlk* b;
    int a0, a1, dim;
  };
  std::map<QN, std::map<std::pair<int, int>, std::vector<Entry>>> bycol;  // q -> traced part -> psi blocks
  for (const PsiBlk& b : O.blocks) {
    int a0, a1, dim;
    const QN q = key_of(b, &a0, &a1, &dim);
    const int n1 = b.e / 4, n2 = b.e % 4;
    const std::pair<int, int> c = direction == 0 ? std::make_pair(n2, b.ir) : std::make_pair(b.il, n1);
    bycol[q][c].push_back({&b, a0, a1, dim});
  }
  GemmList gl;
  for (const Sec& s : secs) {
    const auto& rv = rows[s.q];
    for (const RowBlk& ra : rv)
      for (const RowBlk& rb : rv) {
        gl.begin(ra.dim, rb.dim, 1, rbuf, s.rho_off + (int64_t)ra.off * s.n + rb.off, s.n, 0, false);
        for (const auto& cv : bycol[s.q]) {
          const Entry *ea = nullptr, *eb = nullptr;
          for (const Entry& e : cv.second) {
            if (e.a0 == ra.a0 && e.a1 == ra.a1) ea = &e;
            if (e.a0 == rb.a0 && e.a1 == rb.a1) eb = &e;
          }
          if (!ea || !eb) continue;
          if (direction == 0) {
            // psi(a, c) is d_a x d_r (row-major): op(A) = psi(a,c), op(B) = psi(b,c)^T, K = d_r
            GContrib c = make_contrib(ea->b->dr, GF_TRANS_B, 0, ea->b->off, ea->b->dr, 0, eb->b->off, eb->b->dr, 1.0);
            gl.add(c);
          } else {
            // psi(c, a) is d_l x d_a: op(A) = psi(c,a)^T, op(B) = psi(c,b), K = d_l
            GContrib c = make_contrib(ea->b->dl, GF_TRANS_A, 0, ea->b->off, ea->b->dr, 0, eb->b->off, eb->b->dr, 1.0);
            gl.add(c);
          }
        }
        gl.end();
      }
  }
  std::vector<double> hw((size_t)w_total), hvec;
  std::vector<int> hinfo(secs.size(), 0);
  auto cleanup = [&]() {
    dev_free(rho);
    dev_free(w);
    dev_free(work);
    dev_free(info);
  };
  try {
    if (!gl.tasks.empty()) {
      gl.upload();
      gl.run(tab, psi, nullptr, P_F64, stream);
    }
    for (size_t i = 0; i < secs.size(); ++i)
      dev_syevd(rho + secs[i].rho_off, secs[i].n, secs[i].n, w + secs[i].w_off, work, info + i, stream);
    dev_d2h(hw.data(), w, sizeof(double) * (size_t)w_total, stream);
    dev_d2h(hinfo.data(), info, sizeof(int) * secs.size(), stream);
    for (size_t i = 0; i < secs.size(); ++i)
      DMRG_CHECK(hinfo[i] == 0, DMRG_EINTERNAL, "reduced density matrix eigensolver did not converge");
    // states by descending weight (ties: sector order, then eigenvector index)
    struct St {
      double lam;
      int s, j;
    };
    std::vector<St> all;
    double total = 0;
    for (int i = 0; i < (int)secs.size(); ++i)
      for (int j = 0; j < secs[i].n; ++j) {
        const double lam = std::max(0.0, hw[secs[i].w_off + j]);
        total += lam;
        all.push_back({lam, i, j});
      }
    DMRG_CHECK(total > 0 && std::isfinite(total), DMRG_EINVAL, "psi is zero or not finite");
    std::stable_sort(all.begin(), all.end(), [](const St& x, const St& y) {
      if (x.lam != y.lam) return x.lam > y.lam;
      if (x.s != y.s) return x.s < y.s;
      return x.j > y.j;
    });
    std::vector<std::vector<int>> kept(secs.size());  // eigenvector columns, descending weight
    double kept_w = 0, entropy = 0;
    for (const St& st : all) {
      if ((int)(&st - all.data()) >= D) break;
      if (cutoff > 0 && st.lam <= cutoff * total) break;
      kept[st.s].push_back(st.j);
      kept_w += st.lam;
      const double p = st.lam / total;
      entropy -= p * std::log(p);
    }
    hvec.resize((size_t)rho_total);
    dev_d2h(hvec.data(), rho, sizeof(double) * (size_t)rho_total, stream);

    auto R = std::make_unique<Decimation>();
    R->direction = direction;
    R->discarded = std::max(0.0, (total - kept_w) / total);
    R->entropy = entropy;
    std::vector<int> new_index(secs.size(), -1);
    for (int i = 0; i < (int)secs.size(); ++i)
      if (!kept[i].empty()) {
        new_index[i] = (int)R->sec.size();
        R->sec.push_back(secs[i].q);
        R->dim.push_back((int)kept[i].size());
      }
    DMRG_CHECK(!R->sec.empty(), DMRG_EINVAL, "no state kept (cutoff too large)");
    // the new site tensor, blocks in the dmrg_mps enumeration order; a block
    // whose rows do not occur in psi holds zeros
    auto put_block = [&](int si, const RowBlk* rb, int rows_, int cols_, bool rows_are_states) {
      const Sec& s = secs[si];
      const double* V = hvec.data() + s.rho_off;  // column-major eigenvectors
      R->blk_off.push_back((int64_t)R->data.size());
      const size_t base = R->data.size();
      R->data.resize(base + (size_t)rows_ * cols_, 0.0);
      if (!rb) return;
      for (int r = 0; r < rows_; ++r)
        for (int c = 0; c < cols_; ++c) {
          const int state = rows_are_states ? r : c, elem = rows_are_states ? c : r;
          const int j = kept[si][state];
          R->data[base + (size_t)r * cols_ + c] = V[(int64_t)(rb->off + elem) + (int64_t)j * s.n];
        }
    };
    if (direction == 0) {
      // A[k]: blocks (il at bond k, n, iq at bond k+1), il then n ascending
      for (int il = 0; il < (int)O.Llabel.size(); ++il)
        for (int n = 0; n < 4; ++n) {
          const QN q = O.Llabel[il] + SITE_QN[n];
          auto it = sec_index.find(q);
          if (it == sec_index.end() || new_index[it->second] < 0) continue;
          put_block(it->second, row_index(q, il, n), O.Lb.dim[il], (int)kept[it->second].size(), false);
        }
    } else {
      // A[k+1]: blocks (iq at bond k+1, n, ir at bond k+2), iq then n ascending
      for (int si = 0; si < (int)secs.size(); ++si) {
        if (new_index[si] < 0) continue;
        for (int n = 0; n < 4; ++n) {
          const QN qr = secs[si].q + SITE_QN[n];
          int ir = -1;
          for (int t = 0; t < (int)O.Rlabel.size(); ++t)
            if (O.Rlabel[t] == qr) ir = t;
          if (ir < 0) continue;
          put_block(si, row_index(secs[si].q, n, ir), (int)kept[si].size(), O.Rb.dim[ir], true);
        }
      }
    }
    O.decim = std::move(R);
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}

}  // namespace dmrg
