/*
 * dmrg.h -- C ABI of the MI355X two-site DMRG sigma-vector engine.
 *
 * The library computes, for one bond of an ab initio DMRG sweep, the Davidson
 * sigma-vector sigma = H psi of the two-dot problem (paper, Sec. 2.1, Eq. Sigma;
 * Hamiltonian Eq. Hsq, sum-of-products form Eq. totoalH), its diagonal, and
 * the lowest eigenpair by Davidson's method.  The renormalized block
 * operators (the qops set, Sec. 2.3, Eq. qops) are built on the GPU from the
 * integrals and a U(1)xU(1) block-sparse MPS (Eq. MPS, Eq. Renorm).
 *
 * Conventions
 *   - Spatial orbitals 0..K-1, one per site, in MPS order.  Spin orbital
 *     p = 2*i + s (s = 0 alpha, 1 beta); Jordan-Wigner order is site by site,
 *     alpha before beta.  Site basis n = 0..3 is {|vac>, |beta>, |alpha>,
 *     |alpha beta>} (Sec. 2.1) with |alpha beta> = a+_alpha a+_beta |vac>.
 *   - Bond b (0..K) lies between sites b-1 and b.  A sector at bond b is
 *     labelled by (q_alpha, q_beta), the electron numbers of sites 0..b-1.
 *   - All functions return 0 on success or a negative dmrg_status; nothing
 *     throws across the ABI.  dmrg_last_error() gives a message.
 *   - All floating point data are IEEE binary64 unless stated otherwise.
 *   - Every entry point that takes a context issues its GPU work on the
 *     context's HIP stream, in call order.  Calls that share a context must
 *     not run concurrently from several host threads.
 *   - An operator handle (dmrg_ops) is not read-only: sigma, diag, Davidson
 *     and the preconditioner calls reuse scratch it owns (the R-step buffers,
 *     FP32 operator copies, work counters).  Calls on one handle are ordered
 *     on the GPU even across contexts: a call on a stream other than the
 *     handle's previous one first makes its stream wait for the previous
 *     call's work.  Calls on one handle must still not be made concurrently
 *     from several host threads.
 */
#ifndef DMRG_H
#define DMRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DMRG_OK = 0,
  DMRG_EINVAL = -1,   /* bad argument (null pointer, out-of-range value) */
  DMRG_ESHAPE = -2,   /* inconsistent sectors / MPS blocks / empty two-dot space */
  DMRG_ENOMEM = -3,   /* device or host allocation failed */
  DMRG_EHIP = -4,     /* a HIP runtime call or kernel launch failed */
  DMRG_ENOCONV = -5,  /* Davidson reached max_iter; the best pair is still returned */
  DMRG_EINTERNAL = -6
} dmrg_status;

typedef enum { DMRG_FP64 = 0, DMRG_FP32 = 1, DMRG_BF16X3 = 2 } dmrg_precision;

typedef struct dmrg_ctx dmrg_ctx;  /* device, stream, last error */
typedef struct dmrg_ops dmrg_ops;  /* renormalized operators + sigma plan of one bond (device) */

/* Integrals of Eq. (Hsq) in spatial orbitals (host memory, read during the call,
 * never retained):
 *   h[K*K]       one-electron h_pq, row-major, symmetric
 *   eri[K^4]     two-electron (pq|rs) in chemist notation, index ((p*K+q)*K+r)*K+s,
 *                with the 8-fold permutational symmetry of real orbitals
 *   ecore        constant added to H (enters sigma as ecore*psi). */
typedef struct {
  int K;
  const double* h;
  const double* eri;
  double ecore;
} dmrg_integrals;

/* Block-sparse MPS (Eq. MPS) under U(1)xU(1) (host memory, copied):
 *   K, n_alpha, n_beta   orbitals and target electron numbers
 *   bond                 the two dots are sites (bond, bond+1), 0 <= bond <= K-2
 *   nsec[K+1]            number of sectors at each bond
 *   sec_qn[2*S]          (q_alpha, q_beta) of every sector, bonds in order, S = sum nsec
 *   sec_dim[S]           sector dimensions (> 0)
 *   blk_off[B]           element offset into data of every site-tensor block
 *   data                 site tensors A[j] for j < bond (left-canonical) and
 *                        j > bond+1 (right-canonical), sites ascending.  The blocks
 *                        of A[j] are (il, n, ir) with il a sector of bond j, n a site
 *                        state, ir the sector of bond j+1 with q(ir) = q(il) + q(n);
 *                        enumerated by il ascending then n ascending, each a dense
 *                        d_il x d_ir row-major array.  B counts all such blocks. */
typedef struct {
  int K, n_alpha, n_beta, bond;
  const int* nsec;
  const int* sec_qn;
  const int* sec_dim;
  const int64_t* blk_off;
  const double* data;
} dmrg_mps;

/* Work statistics of one bond's plan (filled by dmrg_ops_stats). */
typedef struct {
  int64_t n_psi;          /* length of psi / sigma */
  int64_t n_blocks;       /* psi blocks */
  int64_t n_terms;        /* operator-pair families x members (terms mu of Eq. totoalH) */
  int64_t n_rgemm;        /* GEMMs of the right-operator step (Eq. sigmablk56) */
  int64_t n_lgemm;        /* GEMMs of the left-operator step (Eq. sigmablk78) */
  double flops_sigma;     /* sum 2MNK over all GEMMs of one sigma call */
  double flops_rstep;     /* the part in the right-operator step */
  double flops_lstep;     /* the part in the left-operator step */
  double op_bytes;        /* device bytes of operators kept for sigma */
  double build_seconds;   /* wall time of dmrg_build_ops */
  double build_flops;     /* sum 2MNK of the renormalization GEMMs */
  /* live kernel timing since the last dmrg_profile(ops, 1): HIP events recorded
   * on the context stream around every GEMM launch of dmrg_sigma (FP64) */
  int64_t prof_sigma_calls;
  int64_t prof_launches;
  double prof_gemm_ms;    /* summed duration of those launches */
} dmrg_stats;

/* Davidson options (paper Sec. 2.1 names Davidson's method; details are ours). */
typedef struct {
  double tol_residual;     /* stop when ||H x - theta x||_2 <= tol_residual (default 1e-6) */
  int max_iter;            /* sigma calls, default 200 */
  int m_max;               /* subspace size before restart, 4..32, default 24 */
  int precision;           /* dmrg_precision of sigma in early iterations */
  double switch_residual;  /* reduced precision used while ||r|| > max(switch_residual,
                              f |theta|), f = 6e-6 (FP32) or 8e-6 (BF16x3): about 2-3 times the
                              largest relative sigma error measured for the format */
  int precond;             /* 0 diagonal, 1 learned MLP (falls back to diagonal) */
  const float* mlp_weights;/* host weights for precond == 1 (dmrg_mlp_nweights floats) */
  double e_ref;            /* if finite: record time/iterations to reach e_ref + e_tol */
  double e_tol;
  int stop_at_ref;         /* nonzero: stop at the first FP64 Ritz value <= e_ref + e_tol */
  int stagnation;          /* switch to FP64 after this many consecutive reduced-precision
                              iterations in which neither ||r|| fell below 0.9x its best nor
                              theta fell by more than 1e-8 |theta| (default 4) */
  double* trace;           /* optional host array [trace_cap][4]: per iteration (seconds since
                              entry, Ritz value, ||r||_2, precision of the sigma behind it) */
  int trace_cap;
  double precond_shift;    /* kappa >= 0: the correction divides by theta - kappa ||r||_2 - H_ii
                              instead of theta - H_ii (default 1; 0 is the plain diagonal
                              preconditioner).  Some eigenvalue lies within ||r||_2 of theta, so
                              theta - ||r||_2 bounds the sought lowest one from below for
                              kappa = 1; the shift keeps the denominators of components with
                              H_ii near theta away from zero.  The learned preconditioner takes
                              the shifted value as its theta (features and base correction). */
} dmrg_davidson_opts;

typedef struct {
  int iterations;          /* sigma calls made */
  int sigma_fp64;          /* of which in FP64 */
  double residual;         /* final ||r||_2 */
  double seconds;          /* wall time of the call */
  double seconds_to_ref;   /* time to first Ritz value <= e_ref + e_tol (or -1) */
  int iters_to_ref;
  int mlp_fallbacks;       /* iterations that used the diagonal correction although
                              precond == 1: after three model steps whose FP64 residual
                              exceeded twice the best one seen (or was not finite) */
  int switch_iter;         /* iteration at which FP64 sigma took over (-1: never reduced) */
  int trace_len;           /* rows written to opts->trace */
} dmrg_davidson_stats;

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t, may be NULL for the default stream). */
int dmrg_create(dmrg_ctx** ctx, int device, void* hip_stream);
void dmrg_destroy(dmrg_ctx* ctx);
const char* dmrg_last_error(const dmrg_ctx* ctx);

/* Scratch budgets and split-k threshold of dmrg_build_ops (0 selects the default). */
typedef struct {
  size_t x_budget_bytes;   /* each of the two R-step scratch slots of sigma (default 16 GiB):
                              a smaller budget splits sigma into more launches */
  size_t t_budget_bytes;   /* renormalization scratch per growth step (default 2 GiB) */
  int64_t ksplit_tiles;    /* sigma's L-step tasks whose k loop is longer than this many
                              k tiles of 32 are split into about equal parts, run as
                              separate jobs and added into sigma, one part after the
                              other, at the end of their launch (default 512; sigma
                              changes with it by rounding only, and never with the
                              launch shape) */
} dmrg_build_opts;

/* Build the renormalized operators of the two-dot problem at mps->bond by
 * growing the left block over sites 0..bond-1 and the right block over sites
 * K-1..bond+2 (Eq. Renorm on the GPU), then form the complementary operators
 * and intermediates and plan sigma.  Synchronous.  opts may be NULL.  *out is
 * owned by the caller and released with dmrg_ops_destroy. */
int dmrg_build_ops(dmrg_ctx* ctx, const dmrg_integrals* ints, const dmrg_mps* mps,
                   const dmrg_build_opts* opts, dmrg_ops** out);
void dmrg_ops_destroy(dmrg_ops* ops);

/* psi layout: the symmetry blocks of the two-dot wavefunction Psi^{l c1 c2 r}
 * (Eq. Sigma; stored blockwise as in Sec. 2.2, where each block is a matrix in
 * C order): blocks (il, n1, n2, ir), il a sector of bond `bond`, ir the sector
 * of bond `bond+2` with q(ir) = q(il) + q(n1) + q(n2), enumerated by (il, n1, n2);
 * each block d_il x d_ir row-major.  blk_meta[6*nb] = (il, n1, n2, ir, d_il, d_ir),
 * blk_off[nb] = element offsets.  Either array may be NULL. */
int dmrg_ops_layout(const dmrg_ops* ops, int64_t* n_psi, int64_t* n_blocks,
                    int* blk_meta, int64_t* blk_off);
int dmrg_ops_stats(const dmrg_ops* ops, dmrg_stats* st);

/* Enable (1) or disable (0) per-launch kernel timing of dmrg_sigma and reset
 * its counters.  While enabled every dmrg_sigma call synchronises the context
 * stream once at its end to read the events. */
int dmrg_profile(dmrg_ops* ops, int enable);

/* sigma = H psi (Eq. Sigma), psi and sigma device pointers of n_psi elements.
 * precision DMRG_FP64: binary64 in and out.  DMRG_FP32 / DMRG_BF16X3: psi and
 * sigma are still binary64 buffers; the contraction runs in reduced precision
 * with FP32 accumulation.  Asynchronous on the context stream.  psi and sigma
 * must not overlap. */
int dmrg_sigma(dmrg_ctx* ctx, dmrg_ops* ops, const double* psi, double* sigma,
               int precision);

/* Diagonal H_ii of the two-dot Hamiltonian of Eq. Sigma in the psi layout
 * (device output): the Davidson preconditioner's diagonal (the diagonal part
 * of the Hamiltonian that Sec. 3 lists among the steps outside sigma).  It
 * sums the terms of Eq. totoalH whose operators conserve every block's
 * quantum numbers, from the diagonals of their renormalized operators.
 * Synchronous. */
int dmrg_diag(dmrg_ctx* ctx, dmrg_ops* ops, double* diag);

/* dmrg_diag for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  It
 * makes no device allocation: the gathered operator diagonals, the pointer
 * table and the GEMM task lists live in a static 64 MiB device array of the
 * library (one per GPU, set up by dmrg_create on that GPU and held until the
 * process ends).  The members of each operator family are processed in
 * chunks that fit it, so results equal dmrg_diag's to rounding (bit for bit
 * when every family fits one chunk).  Limit: one member's diagonals,
 * 8 * (left + right block dimension) bytes, plus a chunk's task list must fit
 * in 60 MiB; otherwise DMRG_ENOMEM with a message, and diag is unspecified.
 * The scratch keeps the last call's contents.  Calls on one GPU share it:
 * the library serialises them within a process and each call is synchronous
 * (returns when its work on the context stream is done); two processes on one
 * GPU each have their own copy.  diag (device, n_psi) as in dmrg_diag. */
int dmrg_diag_noalloc(dmrg_ctx* ctx, dmrg_ops* ops, double* diag);

/* sigma for nprob independent problems (each its own dmrg_ops, psi and sigma
 * device buffers, psi/sigma as in dmrg_sigma) in one fused launch sequence:
 * launch j runs launch j of every problem's plan, with all problems' tiles in
 * one XCD schedule; the sequence is captured once into a HIP graph and
 * replayed while the ops and pointer sets stay the same (the context keeps
 * the last plan; changing the set rebuilds it).  The first call with a new set
 * also autotunes the launch shapes (a few extra sigma sequences).  Results
 * equal those of dmrg_sigma per problem bit for bit.  flags: DMRG_BATCH_EAGER
 * issues the launches directly instead of through the graph; DMRG_BATCH_NO_TUNE
 * keeps the default shapes.  Asynchronous on the context stream (the first
 * call and calls with new pointers synchronise it). */
#define DMRG_BATCH_EAGER 1
#define DMRG_BATCH_NO_TUNE 2
int dmrg_sigma_batched(dmrg_ctx* ctx, int nprob, dmrg_ops* const* ops,
                       const double* const* psi, double* const* sigma, int precision, int flags);

/* Autotune the launch shapes of dmrg_sigma in one precision: every tile shape
 * of dmrg_launch_shape (64x64, 32x32, 64x32, 32x64, mixed, 128x128, big),
 * each with one workgroup per job and with dynamic units
 * (grid_per_xcd -1), is timed per launch on one sigma call, and the fastest is kept
 * for later calls (results do not change).  Synchronous.  ms_default /
 * ms_tuned (may be NULL) receive the summed launch times with the default
 * and the chosen shapes. */
int dmrg_autotune(dmrg_ctx* ctx, dmrg_ops* ops, int precision, double* ms_default, double* ms_tuned);

/* Launch shapes of dmrg_sigma in one precision, set by hand (what the
 * autotuner otherwise chooses): tile 0 = 64x64, 1 = 32x32, 2 = 64x32,
 * 3 = 32x64 outputs per workgroup, 4 = mixed (64x64 interior, 32-wide strips
 * for at most 32 rows or columns left over, per task), 5 = 128x128 outputs
 * per 1024-thread workgroup, 6 = big (the 128x128-tiled interiors of tasks
 * with long k loops in one launch of 1024-thread workgroups, then everything
 * else cut as in 4 in a second launch); grid_per_xcd > 0 caps
 * the workgroups per XCD (persistent, jobs dealt round robin), 0 = one
 * workgroup per job, -1 = dynamic: the workgroups that fit on the chip at
 * once take cost-balanced ranges of jobs from a per-XCD counter.  Other
 * negative values are DMRG_EINVAL.  Results do not depend on the shape.  The task lists for a new shape are built on first
 * use (synchronous). */
int dmrg_launch_shape(dmrg_ops* ops, int precision, int tile, int64_t grid_per_xcd);

/* Lowest eigenpair.  psi (device, n_psi) holds the initial guess and receives
 * the normalised eigenvector; *energy its FP64 Rayleigh quotient (ecore
 * included).  Synchronous.  opts or stats may be NULL (defaults). */
int dmrg_davidson(dmrg_ctx* ctx, dmrg_ops* ops, double* psi,
                  const dmrg_davidson_opts* opts, double* energy,
                  dmrg_davidson_stats* stats);
void dmrg_davidson_default_opts(dmrg_davidson_opts* opts);

/* ---- Decimation: the truncation step of the two-dot sweep (Sec. 2.1) ----
 *
 * dmrg_decimate splits the two-dot vector psi (device, n_psi, the layout of
 * ops) at the bond between the dots, bond+1.  For every sector q of that
 * bond (electron numbers of sites 0..bond) it forms the reduced density
 * matrix of one side and diagonalises it on the GPU:
 *   direction 0 (sweeping left to right): rows (l, n1), the left block state
 *     and the first dot, with q(l) + q(n1) = q;
 *   direction 1 (right to left): rows (n2, r) with q(r) - q(n2) = q.
 * The eigenvalues are the squared Schmidt coefficients.  The D largest over
 * all sectors are kept (ties: lower sector first); with cutoff > 0 only those
 * whose weight exceeds cutoff * <psi|psi>, with cutoff = 0 zero weights too
 * (so that D >= the full dimension keeps the enlarged block's whole space); their eigenvectors form the new site tensor, in the
 * dmrg_mps format:
 *   direction 0: A[bond], left-canonical, blocks (il at bond, n, iq at bond+1);
 *   direction 1: A[bond+1], right-canonical, blocks (iq at bond+1, n, ir at bond+2);
 * with iq indexing the kept sectors of bond+1 in increasing (q_alpha, q_beta).
 * A block whose rows do not occur in psi is zero.  out receives the sizes,
 * the number of states kept, the discarded weight (weight of the dropped
 * states over <psi|psi>) and the von Neumann entropy of the kept weights.
 * The result stays in ops until the next call; dmrg_decimation_get copies it
 * to caller arrays of out->nsec (sec_qn: 2 ints each, sec_dim), out->nblk
 * (blk_off, offsets into data) and out->ndata (data) entries; any may be
 * NULL.  Synchronous.  DMRG_EINVAL: D < 1, unknown direction, cutoff outside
 * [0, 1), zero psi, or no state kept. */
typedef struct {
  int nsec;
  int kept;
  int64_t nblk;
  int64_t ndata;
  double discarded;
  double entropy;
} dmrg_decimation_info;
int dmrg_decimate(dmrg_ctx* ctx, dmrg_ops* ops, const double* psi, int D, int direction, double cutoff,
                  dmrg_decimation_info* out);
int dmrg_decimation_get(const dmrg_ops* ops, int* sec_qn, int* sec_dim, int64_t* blk_off, double* data);

/* ---- Learned Davidson preconditioner (an addition to the paper's method) ----
 *
 * A Davidson correction is t_i = g_i * d_i: d_i = r_i / (theta - H_ii) is the
 * diagonal correction (|theta - H_ii| floored at 1e-8, sign kept) and the gain
 * g_i = MLP(f_i) is evaluated per psi element by a network of FP32 layers
 * DMRG_MLP_NFEAT -> ReLU(DMRG_MLP_HIDDEN) -> ReLU(DMRG_MLP_HIDDEN) -> 1.
 * Features of element i, in block (il, n1, n2, ir) of a bond with dots at
 * sites (k, k+1), theta the Ritz value and r the residual:
 *   0      clamp((H_ii - theta) / s_h, -8, 8),  s_h = rms over i of (H_ii - theta)
 *   1      asinh((H_ii - theta) / ||r||_2) / 4
 *   2      clamp(r_i / s_r, -8, 8),              s_r = rms over i of r_i
 *   3      log10(||r||_2) / 4
 *   4, 5   (q_alpha, q_beta)(il) - (N_alpha, N_beta) * k / K, over sqrt(K)
 *   6, 7   the right block's electrons (N - q(ir)) - N * (K - k - 2) / K, over sqrt(K)
 *   8..11  one-hot n1;  12..15 one-hot n2
 *   16, 17 log2(d_il) / 10, log2(d_ir) / 10
 * Weights (host float arrays of dmrg_mlp_nweights() entries) in this order:
 * W1[NFEAT][HIDDEN], b1[HIDDEN], W2[HIDDEN][HIDDEN], b2[HIDDEN], w3[HIDDEN], b3
 * (W[in][out], row-major). */
#define DMRG_MLP_NFEAT 18
#define DMRG_MLP_HIDDEN 256

/* Number of floats in a weight vector. */
int dmrg_mlp_nweights(void);

/* Seeded initial weights: uniform(-sqrt(6/fan_in), +) hidden layers, zero
 * biases, w3 = 0 and b3 = 1, so that the initial network is the diagonal
 * preconditioner (g = 1). */
int dmrg_mlp_init(float* weights, uint64_t seed);

/* Training pairs from one bond.  Runs FP64 Davidson with the diagonal
 * preconditioner (default shift) from psi0 (device, n_psi; not modified) for at most max_iter
 * sigma calls and, at every iteration, draws per_iter element indices
 * (seeded) and records for each: the features f_i, the diagonal correction
 * d_i, and the target s*e_i, where e is the part of the reference eigenvector
 * psi_ref (device, normalised) orthogonal to the current Davidson subspace
 * (which holds the Ritz vector) -- the direction the next correction has to
 * supply -- and s = <d,e>/<e,e> is the scale that best matches d.  Host outputs of capacity cap pairs: feat[cap][NFEAT], dcorr[cap],
 * target[cap]; *n_out receives the number written.  Synchronous. */
int dmrg_mlp_collect(dmrg_ctx* ctx, dmrg_ops* ops, const double* psi0, const double* psi_ref,
                     int max_iter, int per_iter, uint64_t seed, int64_t cap, float* feat,
                     float* dcorr, float* target, int64_t* n_out);

/* Fit the gains by Adam with the GPU training kernels, on host inputs of n
 * pairs as written by dmrg_mlp_collect.  group == 0: loss mean_i (g(f_i) d_i -
 * target_i)^2 over minibatches of `batch` pairs.  group > 0: the pairs form
 * groups of `group` consecutive entries (one Davidson iteration each; n a
 * multiple of group) and the loss of a group is 1 - cos^2(g.d, target), the
 * misalignment of the correction with the ideal one, which Davidson's
 * subspace step does not see the scale of; one group per step (batch unused).
 * A seeded tenth of the pairs (groups) is held out, and of the start point and
 * the weights after each epoch the one with the lowest held-out loss is kept.
 * weights (host) are read as the start point and overwritten with the result;
 * loss_before/after (may be NULL) receive the loss over all data.
 * Synchronous. */
int dmrg_mlp_train(dmrg_ctx* ctx, int64_t n, const float* feat, const float* dcorr,
                   const float* target, int group, int epochs, int batch, float lr, uint64_t seed,
                   float* weights, double* loss_before, double* loss_after);

/* One preconditioner application on the device: t = g(f) * d for residual r
 * and diagonal diag (device, n_psi each) at Ritz value theta; weights host. */
int dmrg_mlp_apply(dmrg_ctx* ctx, dmrg_ops* ops, const float* weights, const double* r,
                   const double* diag, double theta, double* t);

#ifdef __cplusplus
}
#endif
#endif
