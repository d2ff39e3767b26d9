// Dry-run device layer for the plan bounds checker (test infrastructure only;
// never part of the product library).
//
// It implements the interface of csrc/device.h on the host without doing any
// arithmetic.  Device allocations get fake addresses in a reserved range, one
// registry entry each, separated by unmapped gaps; host memory backs an
// allocation only once the planner uploads into it (task lists, pointer
// tables, coefficient arrays).  Every kernel entry point checks that each
// byte it would touch lies inside one live allocation, and gemm_launch
// re-derives, from the uploaded task list, the byte range and the 32-bit
// buffer offsets of every operand tile, output tile and scale read of every
// task, the partition of every task's tiles into XCD pieces, the XCD job
// numbering, the bucket lookup of every job and the dynamic unit table,
// following the grouped GEMM kernel's addressing.  A violation throws.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <vector>

#include "../../paper_2311_02854_amd/csrc/common.h"
#include "../../paper_2311_02854_amd/csrc/device.h"

namespace dmrg {

namespace {

constexpr uint64_t BASE = uint64_t(1) << 44;  // fake device addresses start here
constexpr uint64_t GAP = uint64_t(1) << 20;   // unmapped bytes between allocations
constexpr int64_t BKC = 32;                   // k tile of the GEMM kernel

struct Alloc {
  uint64_t size;
  std::unique_ptr<char[]> host;  // backing after the first upload
};

std::map<uint64_t, Alloc> g_alloc;
uint64_t g_next = BASE;

struct Stats {
  int64_t launches = 0, tasks = 0, contrib_checks = 0, jobs = 0, bytes_max = 0;
} g_stats;

[[noreturn]] void fail(const std::string& m) { throw Error(DMRG_EINTERNAL, "plancheck: " + m); }

std::string hex(uint64_t a) {
  char b[32];
  std::snprintf(b, sizeof b, "0x%llx", (unsigned long long)a);
  return b;
}

// allocation containing [a, a + n) (n > 0), or failure
std::map<uint64_t, Alloc>::iterator find(uint64_t a, uint64_t n, const char* what) {
  auto it = g_alloc.upper_bound(a);
  if (it == g_alloc.begin()) fail(std::string(what) + ": address " + hex(a) + " below every allocation");
  --it;
  if (a < it->first || a + n > it->first + it->second.size)
    fail(std::string(what) + ": bytes [" + hex(a) + ", +" + std::to_string(n) + ") outside the allocation at " +
         hex(it->first) + " of " + std::to_string(it->second.size) + " bytes");
  return it;
}

void check(const void* p, int64_t lo, int64_t hi_excl, const char* what) {
  if (hi_excl <= lo) return;
  if (!p) fail(std::string(what) + ": null buffer");
  find((uint64_t)p + (uint64_t)lo, (uint64_t)(hi_excl - lo), what);
}

template <typename T>
const T* view(const void* p, size_t count, const char* what) {
  if (count == 0) return nullptr;
  auto it = find((uint64_t)p, count * sizeof(T), what);
  if (!it->second.host) fail(std::string(what) + ": read of device memory the host never wrote");
  return reinterpret_cast<const T*>(it->second.host.get() + ((uint64_t)p - it->first));
}

size_t count_of(const void* p, size_t elem) {
  auto it = find((uint64_t)p, 1, "count");
  return (size_t)((it->first + it->second.size - (uint64_t)p) / elem);
}

}  // namespace

void plancheck_report() {
  std::printf("plancheck: %lld launches, %lld tasks, %lld contribution checks, %lld jobs, %zu live allocations "
              "(the static scratch included)\n",
              (long long)g_stats.launches, (long long)g_stats.tasks, (long long)g_stats.contrib_checks,
              (long long)g_stats.jobs, g_alloc.size());
}

void dev_set(int) {}

int64_t g_nalloc = 0;
int64_t plancheck_alloc_count() { return g_nalloc; }

// the static scratch: one fake allocation, of PLANCHECK_SCRATCH_BYTES if set
static void* g_scratch = nullptr;
size_t scratch_bytes() {
  const char* e = std::getenv("PLANCHECK_SCRATCH_BYTES");
  return e ? (size_t)std::strtoull(e, nullptr, 10) : (size_t(64) << 20);
}
void scratch_init(int) {
  if (!g_scratch) {
    g_scratch = dev_alloc(scratch_bytes());
    --g_nalloc;  // set-up, not a call's allocation
  }
}
void* scratch_get(int) {
  if (!g_scratch) fail("static scratch used before set-up");
  return g_scratch;
}

void* dev_alloc(size_t bytes) {
  ++g_nalloc;
  const uint64_t a = g_next;
  const uint64_t sz = bytes ? bytes : 1;
  g_next += ((sz + 255) & ~uint64_t(255)) + GAP;
  g_alloc[a] = Alloc{sz, nullptr};
  return (void*)a;
}

void* dev_alloc_nozero(size_t bytes) { return dev_alloc(bytes); }
void* host_alloc_pinned(size_t bytes) { return new char[bytes ? bytes : 1]; }
void host_free_pinned(void* p) { delete[] (char*)p; }
void dev_h2d_async(void* dst, const void* src, size_t bytes, void*) { dev_h2d(dst, src, bytes); }
void dev_h2d_on(void* dst, const void* src, size_t bytes, void*) { dev_h2d(dst, src, bytes); }

void dev_free(void* p) {
  if (!p) return;
  auto it = g_alloc.find((uint64_t)p);
  if (it == g_alloc.end()) fail("free of " + hex((uint64_t)p) + ", which is not a live allocation");
  g_alloc.erase(it);
}

void dev_h2d(void* dst, const void* src, size_t bytes) {
  if (!bytes) return;
  auto it = find((uint64_t)dst, bytes, "dev_h2d");
  if (!it->second.host) it->second.host.reset(new char[it->second.size]());
  std::memcpy(it->second.host.get() + ((uint64_t)dst - it->first), src, bytes);
}

void dev_d2h(void* dst, const void* src, size_t bytes, void*) {
  if (!bytes) return;
  auto it = find((uint64_t)src, bytes, "dev_d2h");
  if (it->second.host)
    std::memcpy(dst, it->second.host.get() + ((uint64_t)src - it->first), bytes);
  else
    std::memset(dst, 0, bytes);
}

void dev_sync(void*) {}
void dev_check(const char*) {}
double wall_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}
void* ev_create() { return new int(0); }
void ev_destroy(void* ev) { delete (int*)ev; }
void ev_record(void*, void*) {}
void stream_wait(void*, void*) {}
float ev_elapsed_ms(void*, void*) { return 1.0f; }
void* stream_create() { return new int(0); }
void stream_destroy(void* s) { delete (int*)s; }
void graph_begin(void*) {}
void* graph_end(void*) { return new int(0); }
void graph_launch(void*, void*) {}
void graph_destroy(void* g) { delete (int*)g; }

// ---- the grouped GEMM --------------------------------------------------------

namespace {

// One operand tile of the kernel: ROWS rows starting at r0 of op(X), element
// (r, k) at X + r*sr + k*sk.  Checks (a) the thread offsets of one k tile fit
// the 32-bit arithmetic of the buffer loads, (b) the bytes the descriptor can
// reach for this tile (from the tile's first element to the operand's last
// valid element among its rows) lie in one allocation.
void check_tile(const char* base, int64_t sr, int64_t sk, int r0, int rows, int K, int ROWS, int64_t tsz,
                const char* what) {
  const int64_t span = ((int64_t)(ROWS - 1) * sr + (BKC - 1) * sk + 1) * tsz;
  if (span > 0x7fffffffLL) fail(std::string(what) + ": k-tile thread offsets exceed 32 bits (" +
                                std::to_string(span) + " bytes)");
  int rv = rows - r0;
  rv = rv < ROWS ? rv : ROWS;
  if (rv <= 0 || K <= 0) return;
  const int64_t last = sk == 1 ? (int64_t)(rv - 1) * sr + (K - 1) : (int64_t)(K - 1) * sk + (rv - 1);
  const char* origin = base + (int64_t)r0 * sr * tsz;
  // the descriptor of k tile i starts at origin + i * BK * sk * tsz and ends
  // at origin + (last + 1) * tsz: the union is [origin, origin + (last+1) tsz)
  check(origin, 0, (last + 1) * tsz, what);
  g_stats.bytes_max = std::max<int64_t>(g_stats.bytes_max, (last + 1) * tsz);
}

const char* buf_ptr(const void* const* table, size_t ntab, int id, const void* p0, void* p1, const char* what) {
  if (id == 0) return (const char*)p0;
  if (id == 1) return (const char*)p1;
  if (id < 0 || (size_t)id >= ntab) fail(std::string(what) + ": buffer id " + std::to_string(id) + " out of table");
  if (!table[id]) fail(std::string(what) + ": buffer id " + std::to_string(id) + " is null in the table");
  return (const char*)table[id];
}

}  // namespace

void gemm_launch(const GTask* tasks_dev, int ntasks, const XcdMap& map, const GContrib* contribs_dev,
                 const int* bucket_dev, void* const* table_dev, const void* p0, void* p1, int elem, int tile,
                 int64_t grid_per_xcd, void*) {
  if (ntasks == 0 || map.max_jobs == 0) return;
  if (tile < 0 || tile >= NTILE) fail("unknown tile shape");
  if (tile == TILE_BIG) fail("TILE_BIG is split on the host into TILE_128 and TILE_EDGE launches");
  if (elem != P_F64 && elem != P_F32 && elem != P_BF16X3) fail("unknown precision");
  ++g_stats.launches;
  const int64_t tsz = elem == P_F64 ? 8 : 4;
  const GTask* T = view<GTask>(tasks_dev, (size_t)ntasks, "task list");
  const size_t ncon = count_of(contribs_dev, sizeof(GContrib));
  const GContrib* C = view<GContrib>(contribs_dev, ncon, "contributions");
  const size_t ntab = count_of(table_dev, sizeof(void*));
  const void* const* tab = view<void*>(table_dev, ntab, "pointer table");

  // XCD task ranges, job numbering, pieces, bucket lookup, units
  if (map.task_begin[0] != 0 || map.task_begin[NXCD] != ntasks) fail("XCD task ranges do not cover the list");
  struct Piece {
    int64_t off, n;
  };
  std::map<int, std::vector<Piece>> pieces;  // task identity (contrib_begin) -> job ranges
  std::map<int, int64_t> task_jobs;
  const size_t nbucket = count_of(bucket_dev, sizeof(int));
  const int* bucket = view<int>(bucket_dev, nbucket, "bucket table");
  for (int x = 0; x < NXCD; ++x) {
    const int tb = map.task_begin[x], te = map.task_begin[x + 1];
    if (tb > te) fail("XCD task ranges out of order");
    int64_t jb = 0;
    for (int t = tb; t < te; ++t) {
      if (T[t].job_begin != jb) fail("XCD job numbering has a gap or overlap");
      jb += T[t].njob;
    }
    if (jb != map.njobs[x]) fail("XCD job count mismatch");
    if (map.njobs[x] > map.max_jobs) fail("max_jobs below an XCD's job count");
    if (map.njobs[x] == 0) continue;
    // bucket lookup: the kernel's find_task binary-searches tasks [bk[b],
    // bk[b + 1]] (sorted by job_begin, checked above) for the last one that
    // starts at or before the job, so it is right for every job of bucket b
    // iff the entries bracket the tasks of the bucket's first and last jobs
    const int64_t nb = (map.njobs[x] >> map.shift) + 1;
    if ((size_t)map.bucket_begin[x] + nb + 1 > nbucket) fail("bucket table too short");
    const int* bk = bucket + map.bucket_begin[x];
    int ti = tb;
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t j0 = b << map.shift;
      if (j0 >= map.njobs[x]) break;
      const int64_t j1 = std::min<int64_t>(((b + 1) << map.shift), map.njobs[x]) - 1;
      while (T[ti].job_begin + T[ti].njob <= j0) ++ti;
      const int t0 = ti;
      int t1 = ti;
      while (T[t1].job_begin + T[t1].njob <= j1) ++t1;
      if (bk[b] < tb || bk[b + 1] >= te || bk[b] > t0 || bk[b + 1] < t1)
        fail("bucket " + std::to_string(b) + " does not bracket the tasks of its jobs");
    }
    g_stats.jobs += map.njobs[x];
    if (grid_per_xcd < 0) {
      const int64_t nu = map.nunits[x];
      const size_t nunit_all = count_of(map.units, sizeof(int64_t));
      if (map.unit_begin[x] < 0 || (size_t)(map.unit_begin[x] + nu + 1) > nunit_all) fail("unit table too short");
      const int64_t* U = view<int64_t>(map.units, nunit_all, "unit table") + map.unit_begin[x];
      if (U[0] != 0 || U[nu] != map.njobs[x]) fail("units do not span the XCD's jobs");
      for (int64_t u = 0; u < nu; ++u)
        if (U[u + 1] <= U[u]) fail("empty or decreasing unit");
      check(map.counters, 0, (int64_t)(64 * (NXCD - 1) + 1) * 4, "unit counters");
    }
  }

  // every task: pieces partition its tiles; operand, scale and output ranges
  std::set<int> done;
  for (int ti = 0; ti < ntasks; ++ti) {
    const GTask& t = T[ti];
    const int shape = tile == TILE_EDGE ? t.shape : tile;
    if (shape < 0 || (shape >= TILE_EDGE && shape != TILE_128) || (tile == TILE_128 && t.shape != TILE_128))
      fail("task shape invalid");
    const int BM = tile_rows(shape), BN = tile_cols(shape);
    if (t.M <= 0 || t.N <= 0 || t.nbatch <= 0) fail("empty task in a device list");
    if (t.tiles_m != (t.M + BM - 1) / BM || t.tiles_n != (t.N + BN - 1) / BN) fail("tile counts mismatch");
    const int64_t jobs = (int64_t)t.tiles_m * t.tiles_n * t.nbatch;
    if (t.job_off < 0 || t.njob <= 0 || t.job_off + t.njob > jobs) fail("piece outside its task's jobs");
    pieces[t.contrib_begin].push_back({t.job_off, t.njob});
    task_jobs[t.contrib_begin] = jobs;
    if (!done.insert(t.contrib_begin).second) continue;
    ++g_stats.tasks;
    if (t.contrib_begin < 0 || t.contrib_end < t.contrib_begin || (size_t)t.contrib_end > ncon)
      fail("contribution range outside the array");
    const int64_t bl[2] = {0, (int64_t)t.nbatch - 1};
    const int mr[2] = {0, (t.tiles_m - 1) * BM}, nr[2] = {0, (t.tiles_n - 1) * BN};
    for (int ci = t.contrib_begin; ci < t.contrib_end; ++ci) {
      const GContrib& c = C[ci];
      ++g_stats.contrib_checks;
      if (c.nred <= 0) fail("contribution without members");
      const int64_t tl[2] = {0, (int64_t)c.nred - 1};
      const bool ta = c.flags & GF_TRANS_A, tb = c.flags & GF_TRANS_B;
      for (int64_t b : bl)
        for (int64_t m : tl) {
          if (c.s_buf >= 0) {
            const char* s = buf_ptr(tab, ntab, c.s_buf, p0, p1, "scale");
            const int64_t o = (c.s_off + b * c.s_bstride + m * c.s_rstride) * tsz;
            check(s, o, o + tsz, "scale");
          }
          const char* Bp = buf_ptr(tab, ntab, c.b_buf, p0, p1, "operand B") +
                           (c.b_off + b * c.b_bstride + m * c.b_rstride) * tsz;
          if (c.flags & GF_IDENT_A) {
            // acc(r, c) += B[c*ldb + r] (tb) or B[r*ldb + c], r < M, c < N
            if (t.M > c.K) fail("identity contribution with more rows than its K");
            const int64_t hi = tb ? (int64_t)(t.N - 1) * c.ldb + (t.M - 1) : (int64_t)(t.M - 1) * c.ldb + (t.N - 1);
            check(Bp, 0, (hi + 1) * tsz, "identity operand");
            continue;
          }
          const char* Ap = buf_ptr(tab, ntab, c.a_buf, p0, p1, "operand A") +
                           (c.a_off + b * c.a_bstride + m * c.a_rstride) * tsz;
          for (int r0 : mr)
            check_tile(Ap, ta ? 1 : c.lda, ta ? c.lda : 1, r0, t.M, c.K, BM, tsz, "operand A");
          for (int n0 : nr)
            check_tile(Bp, tb ? c.ldb : 1, tb ? 1 : c.ldb, n0, t.N, c.K, BN, tsz, "operand B");
        }
    }
    // output tiles: rows [m0, min(M, m0 + BM)), columns [n0, min(N, n0 + BN))
    const int64_t osz = (t.accumulate & GT_C64) ? 8 : tsz;
    const char* Cp = (t.accumulate & GT_C64)
                         ? (t.c_buf == 1 ? (const char*)p1 : buf_ptr(tab, ntab, t.c_buf, p0, p1, "output"))
                         : buf_ptr(tab, ntab, t.c_buf, p0, p1, "output");
    for (int64_t b : bl) {
      const int64_t o = (t.c_off + b * t.c_bstride) * osz;
      check(Cp, o, o + ((int64_t)(t.M - 1) * t.ldc + t.N) * osz, "output");
    }
  }
  for (auto& kv : pieces) {
    auto& v = kv.second;
    std::sort(v.begin(), v.end(), [](const Piece& a, const Piece& b) { return a.off < b.off; });
    int64_t at = 0;
    for (const Piece& p : v) {
      if (p.off != at) fail("a task's pieces leave out or repeat tiles");
      at += p.n;
    }
    if (at != task_jobs[kv.first]) fail("a task's pieces do not cover all its tiles");
  }
}

// ---- vector kernels: range checks only ---------------------------------------

void k_copy_segments(const double* src, double* dst, const int64_t* seg_dev, int nseg, void*) {
  if (nseg <= 0) return;
  const int64_t* S = view<int64_t>(seg_dev, 3 * (size_t)nseg, "copy segments");
  for (int i = 0; i < nseg; ++i) {
    if (S[3 * i + 2] <= 0) fail("empty copy segment");
    check(src, S[3 * i] * 8, (S[3 * i] + S[3 * i + 2]) * 8, "copy source");
    check(dst, S[3 * i + 1] * 8, (S[3 * i + 1] + S[3 * i + 2]) * 8, "copy destination");
  }
}

// split-k reduction: every segment's output and partial ranges (binary64)
void reduce_launch(const ReduceSeg* segs_dev, int nseg, void* const* table_dev, void* p1, void*) {
  if (nseg <= 0) return;
  const ReduceSeg* R = view<ReduceSeg>(segs_dev, (size_t)nseg, "reduction segments");
  const size_t ntab = count_of(table_dev, sizeof(void*));
  const void* const* tab = view<void*>(table_dev, ntab, "pointer table");
  for (int i = 0; i < nseg; ++i) {
    const ReduceSeg& r = R[i];
    if (r.n <= 0 || r.nsrc <= 0 || r.src_stride < r.n) fail("reduction segment empty or overlapping partials");
    check(buf_ptr(tab, ntab, r.dst_buf, nullptr, p1, "reduction output"), r.dst_off * 8, (r.dst_off + r.n) * 8,
          "reduction output");
    const char* src = buf_ptr(tab, ntab, r.src_buf, nullptr, p1, "reduction partial");
    for (int64_t s : {int64_t(0), int64_t(r.nsrc - 1)})
      check(src, (r.src_off + s * r.src_stride) * 8, (r.src_off + s * r.src_stride + r.n) * 8, "reduction partial");
  }
}

void k_fill(double* x, double, int64_t n, void*) { check(x, 0, n * 8, "k_fill"); }
void k_zero_bytes(void* p, size_t bytes, void*) { check(p, 0, (int64_t)bytes, "k_zero_bytes"); }
void k_fill_f(float* x, float, int64_t n, void*) { check(x, 0, n * 4, "k_fill_f"); }
void k_d2f(const double* x, float* y, int64_t n, void*) {
  check(x, 0, n * 8, "k_d2f in");
  check(y, 0, n * 4, "k_d2f out");
}
void k_f2d(const float* x, double* y, int64_t n, void*) {
  check(x, 0, n * 4, "k_f2d in");
  check(y, 0, n * 8, "k_f2d out");
}
void k_axpby(double, const double* x, double, double* y, int64_t n, void*) {
  check(x, 0, n * 8, "k_axpby x");
  check(y, 0, n * 8, "k_axpby y");
}
void k_copy(const double* x, double* y, int64_t n, void*) {
  check(x, 0, n * 8, "k_copy x");
  check(y, 0, n * 8, "k_copy y");
}
void k_multidot(const double* V, int64_t ld, int m, const double* x, int64_t n, double* out, double* part, void*) {
  if (m <= 0) return;
  check(V, 0, ((int64_t)(m - 1) * ld + n) * 8, "k_multidot V");
  check(x, 0, n * 8, "k_multidot x");
  check(out, 0, (int64_t)m * 8, "k_multidot out");
  check(part, 0, (int64_t)MULTIDOT_PART * m * 8, "k_multidot part");
}
void k_lincomb(const double* V, int64_t ld, int m, const double* c, int64_t n, double* y, void*) {
  check(V, 0, ((int64_t)(m - 1) * ld + n) * 8, "k_lincomb V");
  check(c, 0, (int64_t)m * 8, "k_lincomb c");
  check(y, 0, n * 8, "k_lincomb y");
}
void k_sub_lincomb(const double* V, int64_t ld, int m, const double* c, int64_t n, double* y, void* s) {
  k_lincomb(V, ld, m, c, n, y, s);
}
void k_small_eigh(const double* G, int ld, int m, double* w, double* Z, void*) {
  check(G, 0, ((int64_t)(m - 1) * ld + m) * 8, "k_small_eigh G");
  check(w, 0, (int64_t)m * 8, "k_small_eigh w");
  check(Z, 0, (int64_t)m * m * 8, "k_small_eigh Z");
}
void k_precond_diag(const double* r, const double* d, const double* theta, double, double* t, int64_t n, void*) {
  check(r, 0, n * 8, "k_precond_diag r");
  check(d, 0, n * 8, "k_precond_diag d");
  check(theta, 0, 8, "k_precond_diag theta");
  check(t, 0, n * 8, "k_precond_diag t");
}
void k_gather_diag(const double* src, const int64_t* meta, int nblk, int64_t sstride, int64_t dstride, int nmem,
                   double* dst, void*) {
  if (nblk <= 0 || nmem <= 0) return;
  const int64_t* M = view<int64_t>(meta, (size_t)nblk * 3, "gather_diag meta");
  for (int b = 0; b < nblk; ++b) {
    const int64_t so = M[3 * b], dim = M[3 * b + 1], dO = M[3 * b + 2];
    if (dim <= 0) continue;
    for (int64_t mem : {int64_t(0), int64_t(nmem - 1)}) {
      check(src, (mem * sstride + so) * 8, (mem * sstride + so + (dim - 1) * dim + dim) * 8, "gather_diag src");
      check(dst, (mem * dstride + dO) * 8, (mem * dstride + dO + dim) * 8, "gather_diag dst");
    }
  }
}
void k_scale(double* y, double, int64_t n, void*) { check(y, 0, n * 8, "k_scale"); }
void dev_syevd(double* A, int n, int lda, double* w, double* work_e, int* info, void*) {
  if (n <= 0) return;
  check(A, 0, ((int64_t)(n - 1) * lda + n) * 8, "dev_syevd A");
  check(w, 0, (int64_t)n * 8, "dev_syevd w");
  check(work_e, 0, (int64_t)n * 8, "dev_syevd work");
  check(info, 0, 4, "dev_syevd info");
}

// The learned preconditioner's kernels are not on the plan paths the checker
// drives; they only have their vector arguments checked.
void k_mlp_scales(const double* r, const double* diag, const double*, int64_t n, double*, double*, void*) {
  check(r, 0, n * 8, "k_mlp_scales r");
  check(diag, 0, n * 8, "k_mlp_scales diag");
}
void k_mlp_apply(const float*, const double* r, const double* diag, const double*, const double*, const int*,
                 const float*, double, double* out, int64_t n, void*) {
  check(r, 0, n * 8, "k_mlp_apply r");
  check(diag, 0, n * 8, "k_mlp_apply diag");
  check(out, 0, n * 8, "k_mlp_apply out");
}
void k_mlp_gather_pairs(const int64_t*, int, const double*, const double*, const double*, const double*,
                        const int*, const float*, const double*, double, double, float*, float*, float*, void*) {}
void k_mlp_train_fwd(const float*, const float*, int64_t, float*, float*, float*, void*) {}
void k_mlp_bwd_out(const float*, const float*, const float*, const float*, const float*, int64_t, float*, float*,
                   void*) {}
void k_mlp_cos_grad(const float*, const float*, const float*, const float*, const float*, int64_t, float*, float*,
                    float*, void*) {}
void k_relu_mask(float*, const float*, int64_t, void*) {}
void k_colsum(const float*, const float*, int64_t, int, float*, void*) {}
void k_sum_f(const float*, int64_t, float*, void*) {}
void k_adam(float*, const float*, float*, float*, int64_t, float, float, float, float, float, float, void*) {}
void k_sqerr(const float*, const float*, const float*, int64_t, float*, void*) {}
void k_gather_rows(const float*, const int*, int64_t, int, float*, void*) {}

}  // namespace dmrg
