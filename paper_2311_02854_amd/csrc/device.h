// Device-side interface: memory, streams and kernel launchers.  Implemented in
// kernels.hip; the planner sources only see this header.
#pragma once
#include <cstddef>
#include <cstdint>

namespace dmrg {

// One output matrix (or a batch of nbatch equally laid-out outputs):
//   C[b] (+)= sum_{c in contribs} sum_{t < nred_c} alpha_c * s_c(b,t) *
//             op(A_c(b,t)) * op(B_c(b,t))
// with X_c(b,t) = buffer(x_buf) + x_off + b*x_bstride + t*x_rstride and
// s_c(b,t) = buffer(s_buf)[s_off + b*s_bstride + t*s_rstride] (1 if s_buf < 0).
// Buffer ids 0 and 1 are the per-launch pointers p0/p1; ids >= 2 index the
// launch's pointer table.
struct GTask {
  int32_t M, N;
  int32_t nbatch;
  int32_t tiles_m, tiles_n;
  int32_t c_buf;
  int32_t ldc;
  int32_t accumulate;
  int32_t shape;      // tile shape of this task in a mixed-shape launch (TILE_*)
  int32_t pad_;
  int64_t c_off, c_bstride;
  int32_t contrib_begin, contrib_end;
  int64_t job_begin;  // first job of this piece in its XCD's job numbering
  int64_t job_off;    // first job (tile x batch, batch-major) of the piece within the task
  int64_t njob;       // jobs of the piece
};

// Workgroups are dispatched round-robin over the XCDs (workgroup i runs on
// XCD i % NXCD); each XCD walks its own task list so that the tiles sharing
// operands meet in one L2.
constexpr int NXCD = 8;
struct XcdMap {
  int32_t task_begin[NXCD + 1];    // task range of each XCD in the device task array
  int32_t bucket_begin[NXCD + 1];  // bucket-table range of each XCD
  int64_t njobs[NXCD];
  int64_t max_jobs;
  int32_t shift;                   // jobs per bucket = 2^shift
  int32_t dynamic;                 // set per launch: resident workgroups take units from a counter
  // Dynamic launches: the jobs of XCD x are cut into nunits[x] units of
  // consecutive jobs; unit u spans jobs [units[unit_begin[x] + u],
  // units[unit_begin[x] + u + 1]).  counters[64 x] counts the units taken
  // on XCD x (zeroed before every launch).
  const int64_t* units;
  unsigned* counters;
  int64_t unit_begin[NXCD];
  int64_t nunits[NXCD];
};

enum : int32_t { GF_TRANS_A = 1, GF_TRANS_B = 2, GF_IDENT_A = 4 };
// GTask::accumulate bits: add to the existing C; C is binary64 whatever the
// operand precision (the sigma output; buffer 1 always is)
enum : int32_t { GT_ACCUM = 1, GT_C64 = 2 };
// Workgroup tile shapes of the grouped GEMM (rows x columns of C).  The
// 64- and 32-wide shapes run on 256-thread workgroups (four per CU); a
// 128 x 128 tile held by one 256-thread workgroup needs so many registers
// that the occupancy drops to 1-2 waves per SIMD, so TILE_128 runs on
// 1024-thread workgroups whose sixteen waves hold the 64 x 64 path's
// per-wave sub-tiles (one workgroup per CU).
// TILE_EDGE: every task is cut into its 64x64-tiled interior and, where the
// rows or columns left over number at most 32, a 32x64 bottom strip, a 64x32
// right strip and a 32x32 corner, all in one launch (per-task shape).
// TILE_BIG: tasks with long k loops keep their 128x128-tiled interior in a
// TILE_128 launch; the rest of them and every other task are cut as in
// TILE_EDGE and run in a second launch right after it.
enum : int {
  TILE_64x64 = 0,
  TILE_32x32 = 1,
  TILE_64x32 = 2,
  TILE_32x64 = 3,
  TILE_EDGE = 4,
  TILE_128 = 5,
  TILE_BIG = 6,
  NTILE = 7
};
inline int tile_rows(int t) { return t == TILE_128 ? 128 : (t == TILE_32x32 || t == TILE_32x64) ? 32 : 64; }
inline int tile_cols(int t) { return t == TILE_128 ? 128 : (t == TILE_32x32 || t == TILE_64x32) ? 32 : 64; }

struct GContrib {
  int32_t K;
  int32_t flags;
  int32_t a_buf, b_buf, s_buf;
  int32_t lda, ldb;
  int32_t nred;
  double alpha;
  int64_t a_off, b_off, s_off;
  int64_t a_bstride, b_bstride, s_bstride;
  int64_t a_rstride, b_rstride, s_rstride;
};

// Reduction of split-k partial outputs (binary64):
//   dst[dst_off + e] += src[src_off + e] + src[src_off + stride + e] + ...
// over nsrc partials added one after the other, e < n.  Buffer ids as in
// GTask (1 is the per-launch p1).
struct ReduceSeg {
  int32_t dst_buf, src_buf;
  int32_t nsrc, pad_;
  int64_t dst_off, src_off, src_stride, n;
};

enum Prec : int { P_F64 = 0, P_F32 = 1, P_BF16X3 = 2 };

// --- runtime -------------------------------------------------------------
void dev_set(int device);
// Static device scratch of the allocation-free entry points: a file-scope
// __device__ array of scratch_bytes() on every device.  scratch_init looks its
// address up on `device` (which must be current) once; scratch_get returns it.
size_t scratch_bytes();
void scratch_init(int device);
void* scratch_get(int device);
void* dev_alloc(size_t bytes);          // zero-filled; throws Error(ENOMEM)
void* dev_alloc_nozero(size_t bytes);   // contents undefined; throws Error(ENOMEM)
void* host_alloc_pinned(size_t bytes);  // page-locked host memory; throws Error(ENOMEM)
void host_free_pinned(void* p);
// asynchronous copy on `stream` from page-locked host memory
void dev_h2d_async(void* dst, const void* pinned_src, size_t bytes, void* stream);
void dev_free(void* p);
void dev_h2d(void* dst, const void* src, size_t bytes);            // synchronous (complete on return)
// synchronous copy ordered on `stream`: after the work queued there before it,
// complete on return (for buffers that kernels on that stream read)
void dev_h2d_on(void* dst, const void* src, size_t bytes, void* stream);
void dev_d2h(void* dst, const void* src, size_t bytes, void* stream);  // synchronous
void dev_sync(void* stream);
void dev_check(const char* where);      // throws Error(EHIP) on a pending error
double wall_seconds();
void* ev_create();
void ev_destroy(void* ev);
void ev_record(void* ev, void* stream);
void stream_wait(void* stream, void* ev);   // later work on stream waits for ev
float ev_elapsed_ms(void* a, void* b);   // both recorded and complete

// streams and graphs: a non-blocking stream of default priority, stream
// capture (thread-local mode) into an executable graph, and its launch
void* stream_create();
void stream_destroy(void* s);
void graph_begin(void* s);
void* graph_end(void* s);                 // returns the executable graph
void graph_launch(void* exec, void* stream);
void graph_destroy(void* exec);

// --- kernels (all asynchronous on `stream`) --------------------------------
// Grouped, batched GEMM over a task list (tasks/contribs in device memory).
// elem: P_F64 (all buffers double) or P_F32 (operand buffers float, FP32 MFMA)
// or P_BF16X3 (float operand buffers, split-bf16 MFMA, FP32 accumulation);
// outputs of tasks flagged GT_C64 are double in every mode.  tile: TILE_*,
// the shape the tasks' tiles_m / tiles_n were counted with.  grid_per_xcd > 0
// caps the workgroups per XCD (persistent launch, jobs dealt round robin);
// grid_per_xcd < 0 launches the workgroups that fit on the chip at once and
// they take the units of map (cost-balanced job ranges) from a per-XCD
// counter; 0 launches one workgroup per job.
// bucket_dev[bucket_begin[x] + b] is the task of XCD x holding its job b << shift
// (clamped to the XCD's last task); it bounds the kernel's job -> task search.
void gemm_launch(const GTask* tasks_dev, int ntasks, const XcdMap& map, const GContrib* contribs_dev,
                 const int* bucket_dev, void* const* table_dev, const void* p0, void* p1, int elem, int tile,
                 int64_t grid_per_xcd, void* stream);
// dst[d + e] = src[s + e] for every triplet (s, d, n) of seg_dev (device
// memory, nseg triplets) and e < n; the destinations must not overlap.
void k_copy_segments(const double* src, double* dst, const int64_t* seg_dev, int nseg, void* stream);
// The segments segs_dev[0 .. nseg) of a split-k reduction (device memory),
// in one launch; segments must not write the same elements.
void reduce_launch(const ReduceSeg* segs_dev, int nseg, void* const* table_dev, void* p1, void* stream);

void k_fill(double* x, double v, int64_t n, void* stream);
void k_zero_bytes(void* p, size_t bytes, void* stream);  // p 8-byte aligned
void k_fill_f(float* x, float v, int64_t n, void* stream);
void k_d2f(const double* x, float* y, int64_t n, void* stream);
void k_f2d(const float* x, double* y, int64_t n, void* stream);
void k_axpby(double a, const double* x, double b, double* y, int64_t n, void* stream);  // y = a x + b y
void k_copy(const double* x, double* y, int64_t n, void* stream);
// out[i] = sum_j V[j*ld + k] * x[k] over k for j < m  (dots of m vectors with x); result on device.
// part: caller-owned device scratch of MULTIDOT_PART * m doubles for the fixed-order partial sums
// (calls that may run concurrently need their own)
constexpr int MULTIDOT_PART = 512;
void k_multidot(const double* V, int64_t ld, int m, const double* x, int64_t n, double* out, double* part,
                void* stream);
// y[k] = sum_j c[j] V[j*ld + k]   (c on device)
void k_lincomb(const double* V, int64_t ld, int m, const double* c, int64_t n, double* y, void* stream);
// y[k] -= sum_j c[j] V[j*ld + k]
void k_sub_lincomb(const double* V, int64_t ld, int m, const double* c, int64_t n, double* y, void* stream);
// Symmetric eigen-decomposition of an n x n matrix in device memory (rocSOLVER
// syevd): A (lda >= n, either storage order: A is symmetric) is overwritten by
// the eigenvectors, stored column-major (column j at A + j*lda), and w[n]
// receives the eigenvalues in ascending order.  Stream-ordered; throws
// Error(EINTERNAL) if the solver did not converge (checked at the next dev_sync
// through *info, an int in device memory).
void dev_syevd(double* A, int n, int lda, double* w, double* work_e, int* info, void* stream);
// Symmetric eigen-decomposition of a small m x m matrix (m <= 32) by cyclic
// Jacobi; writes eigenvalues ascending to w[m] and eigenvectors (columns) to Z.
void k_small_eigh(const double* G, int ld, int m, double* w, double* Z, void* stream);
// diagonal preconditioner t_i = r_i / (theta - d_i) with |theta - d_i| >= floor
void k_precond_diag(const double* r, const double* d, const double* theta, double floor_,
                    double* t, int64_t n, void* stream);
// copy diagonal elements of square blocks: dst[i] for listed (src offset, dim, dst offset)
void k_gather_diag(const double* src, const int64_t* meta, int nblk, int64_t src_stride,
                   int64_t dst_stride, int nmem, double* dst, void* stream);
// scale the per-member coefficient rows etc.: y[i] *= s
void k_scale(double* y, double s, int64_t n, void* stream);
// --- learned preconditioner (mlp.hip) --------------------------------------
// scales[0] = rms(diag - theta), scales[1] = rms(r), scales[2] = ||r||_2; part holds 2*256 doubles
void k_mlp_scales(const double* r, const double* diag, const double* theta, int64_t n, double* part,
                  double* scales, void* stream);
// out_i = g(f_i) * r_i / (theta - diag_i) with the MLP weights w (device)
void k_mlp_apply(const float* w, const double* r, const double* diag, const double* theta, const double* scales,
                 const int* blk, const float* stat, double floor_, double* out, int64_t n, void* stream);
// features, diagonal correction and es*e at m sampled indices
void k_mlp_gather_pairs(const int64_t* idx, int m, const double* r, const double* diag, const double* theta,
                        const double* scales, const int* blk, const float* stat, const double* e, double es,
                        double floor_, float* feat, float* dcorr, float* target, void* stream);
// forward over rows of F[n][NFEAT]; a1/a2 (optional) receive the activations
void k_mlp_train_fwd(const float* w, const float* F, int64_t n, float* a1, float* a2, float* g, void* stream);
void k_mlp_bwd_out(const float* w, const float* g, const float* d, const float* y, const float* a2, int64_t n,
                   float* dout, float* dz2, void* stream);
// direction loss of one group of n samples (one block; see mlp.hip)
void k_mlp_cos_grad(const float* w, const float* g, const float* d, const float* y, const float* a2, int64_t n,
                    float* dout, float* dz2, float* loss, void* stream);
void k_relu_mask(float* dz, const float* a, int64_t n, void* stream);
void k_colsum(const float* X, const float* v, int64_t n, int ncol, float* out, void* stream);
void k_sum_f(const float* x, int64_t n, float* out, void* stream);
void k_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float c1,
            float c2, float eps, void* stream);
void k_sqerr(const float* g, const float* d, const float* y, int64_t n, float* out, void* stream);
void k_gather_rows(const float* src, const int* perm, int64_t n, int width, float* dst, void* stream);

}  // namespace dmrg
