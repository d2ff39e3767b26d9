// Internal host-side types shared by the planner sources (no HIP here).
#pragma once
#include <array>
#include <cstdint>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dmrg.h"

namespace dmrg {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define DMRG_CHECK(cond, code, msg)                         \
  do {                                                      \
    if (!(cond)) throw ::dmrg::Error((code), (msg));        \
  } while (0)

// Electron numbers (alpha, beta).
struct QN {
  int a = 0, b = 0;
  QN() = default;
  QN(int a_, int b_) : a(a_), b(b_) {}
  QN operator+(QN o) const { return {a + o.a, b + o.b}; }
  QN operator-(QN o) const { return {a - o.a, b - o.b}; }
  QN operator-() const { return {-a, -b}; }
  bool operator==(QN o) const { return a == o.a && b == o.b; }
  bool operator!=(QN o) const { return !(*this == o); }
  bool operator<(QN o) const { return a < o.a || (a == o.a && b < o.b); }
  int n() const { return a + b; }
};

// Site basis {vac, beta, alpha, alpha beta}.
static const QN SITE_QN[4] = {QN(0, 0), QN(0, 1), QN(1, 0), QN(1, 1)};

// Charge of one ladder operator on spin orbital p (creator +, annihilator -).
inline QN mode_qn(int p) { return (p & 1) ? QN(0, 1) : QN(1, 0); }

// 4x4 site operator and 16x16 dot operator, row-major, in the site basis and
// the dot basis e = 4*c1 + c2 respectively.
using Mat4 = std::array<double, 16>;
using Mat16 = std::array<double, 256>;

// Basis of a block: sectors with in-block electron numbers.
struct Basis {
  std::vector<QN> qn;
  std::vector<int> dim;
  std::vector<int64_t> off;
  int64_t total = 0;
  int nsec() const { return (int)qn.size(); }
  int find(QN q) const {
    // sectors are few (<= a few hundred); linear scan is fine
    for (int i = 0; i < nsec(); ++i)
      if (qn[i] == q) return i;
    return -1;
  }
  void finish() {
    off.assign(qn.size() + 1, 0);
    for (size_t i = 0; i < qn.size(); ++i) off[i + 1] = off[i] + dim[i];
    total = off.back();
  }
};

// Layout of operators of charge dq on a basis: one dense block per ket
// sector i whose bra sector q(i)+dq exists; blocks row-major d_bra x d_ket.
struct Layout {
  QN dq;
  std::vector<int> bra, ket;     // per block
  std::vector<int64_t> off;      // per block, element offset
  std::vector<int> by_ket;       // ket sector -> block or -1
  std::vector<int> by_bra;       // bra sector -> block or -1
  int64_t size = 0;
  int nblk() const { return (int)bra.size(); }
};

inline Layout make_layout(const Basis& B, QN dq) {
  Layout L;
  L.dq = dq;
  L.by_ket.assign(B.nsec(), -1);
  L.by_bra.assign(B.nsec(), -1);
  for (int i = 0; i < B.nsec(); ++i) {
    int j = B.find(B.qn[i] + dq);
    if (j < 0) continue;
    L.by_ket[i] = (int)L.bra.size();
    L.by_bra[j] = (int)L.bra.size();
    L.bra.push_back(j);
    L.ket.push_back(i);
    L.off.push_back(L.size);
    L.size += (int64_t)B.dim[j] * B.dim[i];
  }
  return L;
}

// Spin-orbital integrals of Eq. (Hsq) derived on the fly from spatial ones.
struct Integrals {
  int K = 0;
  std::vector<double> h, eri;
  double ecore = 0.0;
  int nmodes() const { return 2 * K; }
  double eri_at(int p, int q, int r, int s) const {
    return eri[(((int64_t)p * K + q) * K + r) * K + s];
  }
  // t_pq = h_pq delta(s_p, s_q)
  double t(int p, int q) const {
    if ((p & 1) != (q & 1)) return 0.0;
    return h[(p >> 1) * K + (q >> 1)];
  }
  // <pq|rs> = (pr|qs) delta(s_p,s_r) delta(s_q,s_s)
  double v(int p, int q, int r, int s) const {
    if ((p & 1) != (r & 1) || (q & 1) != (s & 1)) return 0.0;
    return eri_at(p >> 1, r >> 1, q >> 1, s >> 1);
  }
  // <pq||rs> = <pq|rs> - <pq|sr>
  double w(int p, int q, int r, int s) const { return v(p, q, r, s) - v(p, q, s, r); }
};

}  // namespace dmrg
