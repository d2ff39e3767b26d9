// Renormalized block operators (the qops of one block) on the device, and
// their growth by one site (renormalization, Eq. Renorm of the paper).
#pragma once
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "engine.h"

namespace dmrg {

// Operator name: kind and spin-orbital indices.
//   'C' a+_p    'A' a+_p a+_q (p<q)    'B' a+_p a_s    'S' S_p    'H' H
//   'Y' sum_{s<r} <pq||sr> a+_s a+_r  (P_pq = Y_pq^T)
//   'Q' Q_ps    'X' other intermediates (linear combinations)
struct OpKey {
  char kind = 0;
  int p = -1, q = -1;
  bool operator<(const OpKey& o) const {
    if (kind != o.kind) return kind < o.kind;
    if (p != o.p) return p < o.p;
    return q < o.q;
  }
};

// nmem operators sharing charge dq and one layout, stored contiguously
// (member m at dev + m * lay.size).
struct Group {
  QN dq;
  int parity = 0;
  Layout lay;
  std::vector<OpKey> names;
  double* dev = nullptr;
  int buf = -1;       // id in the owning DevTable
  float* dev32 = nullptr;  // reduced-precision copy (sigma operators only)
  int buf32 = -1;
  bool in_arena = false;   // dev is carved from a DeviceArena (not freed here)
  int n() const { return (int)names.size(); }
  int64_t stride() const { return lay.size; }
  // zero-filled on `stream`; from `arena` if given
  void alloc(DevTable& tab, void* stream, DeviceArena* arena = nullptr);
  void free_dev();
};

// Normal-operator groups of a block.
enum GroupId { G_CA, G_CB, G_AAA, G_AAB, G_ABB, G_B0, G_BAB, G_BBA, G_SA, G_SB, G_H, NG };

struct Block {
  bool left = true;
  int nsites = 0;          // sites in the block
  int first_site = 0;      // lowest site index
  Basis basis;             // in-block electron numbers per sector (MPS sector order)
  std::vector<Group> g;    // NG groups
  std::vector<int> ext_a, ext_b;  // external alpha / beta modes, in S member order
  std::unique_ptr<DeviceArena> arena;  // one allocation holding the groups of a grown block
  ~Block() { free_dev(); }
  void free_dev() {
    for (auto& x : g) x.free_dev();
    if (arena) arena->release();
  }
  int member(int gid, OpKey k) const;  // -1 if absent
};

// Site tensor A[j] on the device (blocks (il, n, ir), row-major d_il x d_ir).
struct SiteTensor {
  double* dev = nullptr;
  int buf = -1;
  std::vector<int64_t> off;
  std::vector<int> il, n, ir;
  std::map<std::pair<int, int>, int> by_left;   // (il, n) -> block
  std::map<std::pair<int, int>, int> by_right;  // (ir, n) -> block
  ~SiteTensor() { dev_free(dev); }
};

// Site operators in the basis {vac, beta, alpha, alpha beta}.
namespace site {
Mat4 I();
Mat4 cre(int spin);  // spin 0 alpha, 1 beta
Mat4 ann(int spin);
Mat4 mul(const Mat4& a, const Mat4& b);
Mat4 tr(const Mat4& a);
Mat4 scale(const Mat4& a, double s);
bool zero(const Mat4& a);
int nelec(int n);
}  // namespace site

struct BuildStats {
  double flops = 0;
  int64_t ngemm = 0;
};

struct Builder {
  const Integrals& I;
  DevTable& tab;
  void* stream;
  int Na, Nb;
  BuildStats st;
  size_t scratch_budget = size_t(2) << 30;  // bytes of T scratch per renormalization chunk
  // task lists, pointer tables and one-launch coefficient arrays of the
  // build's many short launches: staged asynchronously (no host wait)
  std::unique_ptr<UploadRing> ring;
  static constexpr size_t RING_BYTES = size_t(256) << 20;
  // intermediates, T scratch and coefficient arrays of one growth step
  DeviceArena step_arena;

  Builder(const Integrals& ints, DevTable& t, void* s, int na, int nb)
      : I(ints), tab(t), stream(s), Na(na), Nb(nb), ring(new UploadRing(RING_BYTES, s)) {}

  std::unique_ptr<Block> vacuum(bool left);
  // grow a left block by site j (= its nsites) or a right block by site j (= first_site-1)
  // (last: the block is kept for sigma; its groups are separate allocations
  // so that single groups can be freed, else they share one)
  std::unique_ptr<Block> grow(const Block& X, int j, const SiteTensor& A, const Basis& newbasis,
                              bool last = false);
  // intermediate group: out[r] = sum_m coef[r][m] * src member m  (same layout as src)
  // (scratch: the result lives in step_arena, valid until the step ends)
  std::unique_ptr<Group> combine(const Group& src, const std::vector<std::vector<double>>& coef,
                                 std::vector<OpKey> names, bool scratch = false);
  void run(GemmList& gl);
};

std::string key_str(const OpKey& k);

}  // namespace dmrg
