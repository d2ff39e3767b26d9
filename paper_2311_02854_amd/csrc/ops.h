// One bond's device-resident operators and its sigma plan.
#pragma once
#include <functional>
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

// Result of the last decimation of a two-dot vector (decimate.cpp): the kept
// sectors of the bond between the dots (sorted by electron numbers) and the
// new site tensor in the dmrg_mps block order.
struct Decimation {
  int direction = 0;
  std::vector<QN> sec;
  std::vector<int> dim;
  std::vector<int64_t> blk_off;
  std::vector<double> data;
  double discarded = 0, entropy = 0;
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
  // split-k partial outputs of the long L-step tasks of one launch (binary64
  // in every precision), added into sigma at the end of that launch
  double* partial = nullptr;
  int pbuf = -1;
  size_t partial_bytes = 0;
  // psi with its blocks grouped by right sector: the R-step's operand
  std::vector<int64_t> perm_off;      // per block: its offset there
  int64_t* perm_seg = nullptr;        // device (src, dst, count) triplets of the gather
  int nperm_seg = 0;
  double* psi_perm = nullptr;
  float* psi_perm32 = nullptr;
  int permbuf = -1;
  // reduced precision (FP32 / BF16x3): FP32 copies of every buffer the plan
  // reads, under the same buffer ids in a second pointer table
  std::vector<int> sigma_bufs;        // buffer ids read or written by the sigma launches
  std::unique_ptr<DevTable> tab32;    // null until the first reduced-precision call
  float* X32[2] = {nullptr, nullptr};
  float* psi32 = nullptr;
  double op_bytes32 = 0;
  // learned preconditioner (built on first use)
  int* mlp_blk = nullptr;             // psi element -> block
  float* mlp_stat = nullptr;          // per block: static features
  double* mlp_part = nullptr;
  double* mlp_scales = nullptr;
  float* mlp_w = nullptr;
  std::vector<float> mlp_w_host;
  // stats
  double flops_r = 0, flops_l = 0, build_seconds = 0, build_flops = 0, op_bytes = 0;
  int64_t ngemm_r = 0, ngemm_l = 0, nterms = 0;
  // launch shapes per precision chosen by the autotuner (default: 64x64 tiles,
  // one workgroup per job); results do not depend on them
  std::vector<int> tile_choice[3];
  std::vector<int64_t> grid_choice[3];
  double tune_ms_default[3] = {0, 0, 0}, tune_ms_best[3] = {0, 0, 0};
  uint64_t serial = 0;                // unique per build (batched plans key on it)
  // live kernel timing (HIP events around every GEMM launch of sigma)
  bool profile = false;
  std::vector<void*> events;
  double prof_ms = 0;
  int64_t prof_launches = 0, prof_calls = 0;

  // ordering across streams: the handle's scratch (R-step slots, FP32
  // copies, unit counters) is reused by every call, so a call on a stream
  // other than the last one waits for the last call's work first
  std::unique_ptr<Decimation> decim;  // last dmrg_decimate result
  void* order_ev = nullptr;
  void* last_stream = nullptr;
  bool used = false;
  void begin_call(void* stream);
  void end_call(void* stream);

  ~Ops();
  int find_block(int il, int e, int ir) const {
    return blk_index[((size_t)il * 16 + e) * Rb.nsec() + ir];
  }
};

struct BuildOptions {
  size_t x_budget = size_t(16) << 30;      // bytes of each R-step scratch slot (fewer, longer launches)
  size_t t_budget = size_t(2) << 30;       // bytes of renormalization scratch
  // L-step tasks whose k loop exceeds this many k tiles (of 32) are split
  // into about equal parts, run as separate jobs (split k)
  int64_t ksplit_tiles = 512;
};

std::unique_ptr<Ops> build_ops(const Integrals& I, int K, int Na, int Nb, int bond, const int* nsec,
                               const int* sec_qn, const int* sec_dim, const int64_t* blk_off,
                               const double* data, void* stream, const BuildOptions& opt);

void sigma_run(Ops& ops, const double* psi, double* sigma, int prec, void* stream);
// Copy psi into ops.psi_perm (its blocks grouped by right sector; and into
// ops.psi_perm32 for a reduced precision) before the sigma launches.
void gather_psi(Ops& ops, const double* psi, int prec, void* stream);
// Time every tile shape (then a persistent grid) on every launch of one sigma
// call in precision prec and keep the fastest per launch.  Synchronous.
void sigma_autotune(Ops& ops, int prec, void* stream);

// Autotuner core shared with the batched plan: run_all(tile_of_launch,
// grid_of_launch, ms_out) issues one full sigma sequence and returns per-launch
// milliseconds; the tuner picks the fastest shape per launch.
void autotune_launches(size_t nl, const std::function<void(const std::vector<int>&, const std::vector<int64_t>&,
                                                           std::vector<double>&)>& run_all,
                       std::vector<int>& tiles, std::vector<int64_t>& grids, double& ms_default, double& ms_best);
void diag_run(Ops& ops, double* diag, void* stream);
// diag(H) without allocating: operator diagonals, pointer table and GEMM task
// lists live in `scratch` (cap bytes of device memory), members in chunks that
// fit it.  Synchronous.  Throws ENOMEM if one member's diagonals and the task
// list of one chunk do not fit.
void diag_run_noalloc(Ops& ops, double* diag, void* stream, void* scratch, size_t cap);
// FP32 copies of the sigma operators (idempotent; synchronous)
void make_reduced_copies(Ops& ops, void* stream);

// Called by Davidson every iteration with the Ritz vector x, residual r,
// diag(H), the Ritz value (device scalar) and the current subspace (m
// orthonormal vectors of n_psi elements, V[j * n_psi + i]), before the
// correction step.
using DavidsonHook = std::function<void(const double* x, const double* r, const double* diag,
                                        const double* theta_dev, const double* V, int m, int iter)>;
int davidson_run(Ops& O, double* psi, const dmrg_davidson_opts& opt, double* energy, dmrg_davidson_stats* st,
                 void* stream, const DavidsonHook& hook = DavidsonHook());

// keep the D most important states of psi at the bond between the dots
// (direction 0: left side, new A[k]; 1: right side, new A[k+1]); result in
// O.decim.  Synchronous.
void decimate_run(Ops& O, const double* psi, int D, int direction, double cutoff, void* stream);

// learned preconditioner (mlp.cpp)
int mlp_nweights();
void mlp_init(float* w, uint64_t seed);
void mlp_prepare(Ops& O, void* stream);
void mlp_precondition(Ops& O, const double* r, const double* diag, const double* theta_dev, double* t,
                      const float* weights, void* stream);
void mlp_apply_once(Ops& O, const float* weights, const double* r, const double* diag, double theta, double* t,
                    void* stream);
int64_t mlp_collect(Ops& O, const double* psi0, const double* psi_ref, int max_iter, int per_iter, uint64_t seed,
                    int64_t cap, float* feat, float* dcorr, float* target, void* stream);
void mlp_train(int64_t n, const float* feat, const float* dcorr, const float* target, int group, int epochs,
               int batch, float lr, uint64_t seed, float* weights, double* loss_before, double* loss_after,
               void* stream);

}  // namespace dmrg
