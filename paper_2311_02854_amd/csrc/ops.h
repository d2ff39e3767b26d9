// One bond's device-resident operators and its sigma plan.
#pragma once
#include <memory>
#include <string>
#include <vector>

#include "blocks.h"

namespace dmrg {

// psi block (il, e = 4*n1 + n2, ir)
struct PsiBlk {
  int il, e, ir, dl, dr;
  int64_t off;
};

// One family of operator triples O^L . O^D . O^R (Eq. totoalH) with `count`
// members sharing the dot operator D (16x16 in the basis e = 4*c1 + c2).
struct SFam {
  const Group* L = nullptr;  // nullptr: identity on the left block
  int Lbase = 0;
  bool Lt = false;
  const Group* R = nullptr;  // nullptr: identity on the right block
  int Rbase = 0;
  bool Rt = false;
  int count = 1;
  Mat16 D{};
  int piD = 0, piR = 0;      // parities of the dot and right-block factors
  double coef = 1.0;
  const char* tag = "";
};

struct Ops {
  int K = 0, Na = 0, Nb = 0, bond = 0, device = 0;
  double ecore = 0;
  Integrals ints;
  Basis Lb, Rb;                       // in-block electron numbers
  std::vector<QN> Llabel, Rlabel;     // MPS sector labels at bonds k and k+2
  std::unique_ptr<Block> L, R;
  std::vector<std::unique_ptr<Group>> extra;  // complementary operators and intermediates
  std::unique_ptr<DevTable> tab;
  std::vector<PsiBlk> blocks;
  std::vector<int> blk_index;         // il*16*nR + e*nR + ir -> block or -1
  int64_t npsi = 0;
  std::vector<SFam> fams;
  // GEMM launches of one sigma call: R-step X = psi . (O^R)^T (Eq. sigmablk56)
  // and L-step sigma += c zeta D O^L . X (Eqs. sigmablk78, sigmablk fused)
  std::vector<GemmList> launches;
  double* X[2] = {nullptr, nullptr};  // R-step scratch (two slots)
  int Xbuf[2] = {-1, -1};
  size_t Xbytes = 0;
  float* X32 = nullptr;               // reduced-precision scratch
  float* psi32 = nullptr;
  float* sig32 = nullptr;
  bool have32 = false;
  // stats
  double flops_r = 0, flops_l = 0, build_seconds = 0, build_flops = 0, op_bytes = 0;
  int64_t ngemm_r = 0, ngemm_l = 0, nterms = 0;
  // live kernel timing (HIP events around every GEMM launch of sigma)
  bool profile = false;
  std::vector<void*> events;
  double prof_ms = 0;
  int64_t prof_launches = 0, prof_calls = 0;

  ~Ops();
  int find_block(int il, int e, int ir) const {
    return blk_index[((size_t)il * 16 + e) * Rb.nsec() + ir];
  }
};

struct BuildOptions {
  size_t x_budget = size_t(4) << 30;       // bytes of R-step scratch
  size_t t_budget = size_t(2) << 30;       // bytes of renormalization scratch
};

std::unique_ptr<Ops> build_ops(const Integrals& I, int K, int Na, int Nb, int bond, const int* nsec,
                               const int* sec_qn, const int* sec_dim, const int64_t* blk_off,
                               const double* data, void* stream, const BuildOptions& opt);

void sigma_run(Ops& ops, const double* psi, double* sigma, int prec, void* stream);
void diag_run(Ops& ops, double* diag, void* stream);
void make_reduced_copies(Ops& ops, void* stream);

}  // namespace dmrg
