// Host-side helpers around the grouped GEMM kernel: a device pointer table
// and a task-list builder.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "common.h"
#include "device.h"

namespace dmrg {

// Staging for streams of short launches (the operator build): task lists,
// pointer tables and coefficient arrays are copied asynchronously on the
// stream from a page-locked host ring into a device ring, so the host never
// waits for the GPU to upload the next launch.  A copy stays valid until the
// ring wraps; the ring then synchronises the stream first (no launch still
// reads it) and bumps its generation, which invalidates cached copies.
class UploadRing {
 public:
  UploadRing(size_t cap, void* stream) : cap_(cap), stream_(stream) {
    dev_ = (char*)dev_alloc_nozero(cap_);
    try {
      host_ = (char*)host_alloc_pinned(cap_);
    } catch (...) {
      dev_free(dev_);
      throw;
    }
  }
  ~UploadRing() {
    dev_sync(stream_);
    dev_free(dev_);
    host_free_pinned(host_);
  }
  UploadRing(const UploadRing&) = delete;
  UploadRing& operator=(const UploadRing&) = delete;
  // Stage a copy (issued by the next flush(); put() = stage + flush).
  void* stage(const void* src, size_t bytes) {
    const size_t b = ((bytes ? bytes : 1) + 255) & ~size_t(255);
    DMRG_CHECK(b <= cap_, DMRG_ENOMEM, "upload of " + std::to_string(bytes) + " bytes exceeds the staging ring");
    if (head_ + b > cap_) {
      flush();
      dev_sync(stream_);
      head_ = pending_ = 0;
      ++gen_;
    }
    if (bytes) std::memcpy(host_ + head_, src, bytes);
    void* p = dev_ + head_;
    head_ += b;
    return p;
  }
  void flush() {
    if (head_ > pending_) dev_h2d_async(dev_ + pending_, host_ + pending_, head_ - pending_, stream_);
    pending_ = head_;
  }
  void* put(const void* src, size_t bytes) {
    void* p = stage(src, bytes);
    flush();
    return p;
  }
  uint64_t generation() const { return gen_; }

 private:
  char* dev_ = nullptr;
  char* host_ = nullptr;
  size_t cap_, head_ = 0, pending_ = 0;  // [pending_, head_) staged, not yet copied
  uint64_t gen_ = 0;
  void* stream_;
};

// Device memory for short-lived buffers of one step (the operator build's
// intermediates and scratch): carved from large chunks, released all at
// once by reset(), which keeps one chunk as large as all the step used so
// that the next step needs no allocation (a hipMalloc or hipFree of a large
// buffer costs about a millisecond).  reset() and release() may only be
// called once no launch still uses the memory.
class DeviceArena {
 public:
  DeviceArena() = default;
  ~DeviceArena() { release(); }
  DeviceArena(const DeviceArena&) = delete;
  DeviceArena& operator=(const DeviceArena&) = delete;
  void* take(size_t bytes) {
    const size_t b = ((bytes ? bytes : 1) + 255) & ~size_t(255);
    if (chunks_.empty() || head_ + b > chunks_.back().second) {
      const size_t last = chunks_.empty() ? 0 : chunks_.back().second;
      const size_t cap = std::max(b, std::max(2 * last, size_t(64) << 20));
      chunks_.push_back({(char*)dev_alloc_nozero(cap), cap});
      head_ = 0;
    }
    void* p = chunks_.back().first + head_;
    head_ += b;
    return p;
  }
  // one chunk of exactly `bytes` (256-aligned pieces must fit), before any take
  void reserve(size_t bytes) {
    DMRG_CHECK(chunks_.empty(), DMRG_EINTERNAL, "reserve on a used arena");
    const size_t cap = (bytes + 255) & ~size_t(255);
    chunks_.push_back({(char*)dev_alloc_nozero(cap ? cap : 256), cap ? cap : 256});
    head_ = 0;
  }
  void reset() {
    if (chunks_.size() > 1) {
      size_t total = 0;
      for (auto& c : chunks_) total += c.second;
      release();
      chunks_.push_back({(char*)dev_alloc_nozero(total), total});
    }
    head_ = 0;
  }
  void release() {
    for (auto& c : chunks_) dev_free(c.first);
    chunks_.clear();
    head_ = 0;
  }

 private:
  std::vector<std::pair<char*, size_t>> chunks_;
  size_t head_ = 0;
};

// Table of device pointers addressed by buffer id (ids 0 and 1 are the
// per-launch pointers p0 / p1 of gemm_launch).
class DevTable {
 public:
  DevTable() : ptrs_{nullptr, nullptr} {}
  ~DevTable() { dev_free(dev_); }
  DevTable(const DevTable&) = delete;
  DevTable& operator=(const DevTable&) = delete;
  // ids released by set(id, nullptr) are handed out again (ids 0 and 1 are
  // the per-launch pointers)
  int add(void* p) {
    dirty_ = dirty_ring_ = true;
    if (!free_.empty()) {
      const int id = free_.back();
      free_.pop_back();
      ptrs_[id] = p;
      return id;
    }
    ptrs_.push_back(p);
    return (int)ptrs_.size() - 1;
  }
  void set(int id, void* p) {
    if (!p && ptrs_[id] && id >= 2) free_.push_back(id);
    ptrs_[id] = p;
    dirty_ = dirty_ring_ = true;
  }
  void* get(int id) const { return ptrs_[id]; }
  int size() const { return (int)ptrs_.size(); }
  void* const* device() {
    if (dirty_ || ptrs_.size() > cap_) {
      if (ptrs_.size() > cap_) {
        dev_free(dev_);
        cap_ = ptrs_.size() * 2 + 16;
        dev_ = (void**)dev_alloc(cap_ * sizeof(void*));
      }
      dev_h2d(dev_, ptrs_.data(), ptrs_.size() * sizeof(void*));
      dirty_ = false;
    }
    return dev_;
  }
  // a copy of the table in the staging ring (kept while the table and the
  // ring's generation are unchanged)
  void* const* device(UploadRing& ring) {
    if (dirty_ring_ || !ring_copy_ || ring_gen_ != ring.generation()) {
      ring_copy_ = (void**)ring.put(ptrs_.data(), ptrs_.size() * sizeof(void*));
      ring_gen_ = ring.generation();
      dirty_ring_ = false;
    }
    return ring_copy_;
  }

 private:
  std::vector<void*> ptrs_;
  std::vector<int> free_;
  void** ring_copy_ = nullptr;
  uint64_t ring_gen_ = 0;
  bool dirty_ring_ = true;
  void** dev_ = nullptr;
  size_t cap_ = 0;
  bool dirty_ = true;
};

// Bump allocator over caller-provided device memory: places the arrays of a
// task list without allocating (the allocation-free entry points).
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  void* take(size_t bytes) {
    const size_t off = (used + 255) & ~size_t(255);
    DMRG_CHECK(off + bytes <= cap, DMRG_ENOMEM,
               "static scratch too small: needs more than its " + std::to_string(cap) + " bytes");
    used = off + bytes;
    return base + off;
  }
  void reset() { used = 0; }
};

// A list of GEMM tasks executed by one gemm_launch.  The host list is tile
// independent; upload(tile) counts the tasks' tiles for one workgroup tile
// shape, splits them into pieces and assigns the pieces to XCDs.  One device
// copy per tile shape can be kept (they share the contribution array).
class GemmList {
  struct Dev;  // one device copy of the lists (defined below)

 public:
  int tile = TILE_64x64;       // shape used by run()
  int64_t grid_per_xcd = 0;    // > 0: persistent launch with this many workgroups per XCD; < 0: dynamic units
  std::vector<GTask> tasks;
  std::vector<GContrib> contribs;
  std::vector<ReduceSeg> reduce;  // split-k partials added after the GEMM launch(es)
  int64_t njobs = 0;           // jobs at 64x64 tiles (for reporting)
  double flops = 0;
  int64_t ngemm = 0;

  ~GemmList() { release(); }
  GemmList() = default;
  GemmList(const GemmList&) = delete;
  GemmList& operator=(const GemmList&) = delete;
  GemmList(GemmList&& o) noexcept { *this = std::move(o); }
  GemmList& operator=(GemmList&& o) noexcept {
    if (this != &o) {
      release();
      tile = o.tile;
      grid_per_xcd = o.grid_per_xcd;
      tasks = std::move(o.tasks);
      contribs = std::move(o.contribs);
      reduce = std::move(o.reduce);
      dreduce_ = o.dreduce_;
      o.dreduce_ = nullptr;
      nreduce_dev_ = o.nreduce_dev_;
      o.nreduce_dev_ = 0;
      njobs = o.njobs;
      flops = o.flops;
      ngemm = o.ngemm;
      dcontribs_ = o.dcontribs_;
      o.dcontribs_ = nullptr;
      ncontribs_dev_ = o.ncontribs_dev_;
      for (int t = 0; t < NTILE; ++t) {
        dev_[t] = o.dev_[t];
        o.dev_[t] = Dev{};
      }
      rest_ = o.rest_;
      o.rest_ = Dev{};
      big_uploaded_ = o.big_uploaded_;
      o.big_uploaded_ = false;
    }
    return *this;
  }

  void begin(int M, int N, int nbatch, int c_buf, int64_t c_off, int ldc, int64_t c_bstride, bool accumulate) {
    GTask t{};
    t.M = M;
    t.N = N;
    t.nbatch = nbatch;
    t.tiles_m = (M + 63) / 64;
    t.tiles_n = (N + 63) / 64;
    t.c_buf = c_buf;
    t.ldc = ldc;
    t.accumulate = (accumulate ? GT_ACCUM : 0) | (c_buf == 1 ? GT_C64 : 0);
    t.c_off = c_off;
    t.c_bstride = c_bstride;
    t.contrib_begin = t.contrib_end = (int32_t)contribs.size();
    tasks.push_back(t);
  }
  void add(const GContrib& c) {
    GTask& t = tasks.back();
    contribs.push_back(c);
    t.contrib_end = (int32_t)contribs.size();
    if (!(c.flags & GF_IDENT_A)) {
      flops += 2.0 * t.M * (double)t.N * c.K * (double)t.nbatch * c.nred;
      ngemm += (int64_t)t.nbatch * c.nred;
    }
  }
  // Drop the last task if it has no contributions and does not overwrite.
  void end() {
    GTask& t = tasks.back();
    if (t.M <= 0 || t.N <= 0 || t.nbatch <= 0 ||
        (t.contrib_begin == t.contrib_end && (t.accumulate & GT_ACCUM))) {
      contribs.resize(t.contrib_begin);
      tasks.pop_back();
      return;
    }
    t.job_begin = njobs;
    njobs += (int64_t)t.tiles_m * t.tiles_n * t.nbatch;
  }
  bool empty() const { return tasks.empty() && ncontribs_dev_ == 0 && !any_dev(); }

  // Estimated MFMA work of one job of task t at tile shape `tl` (k steps x
  // active 16x16 sub-tiles of the workgroup).
  static double job_cost(const GTask& t, const GContrib* cs, int tl) {
    if (tl == TILE_EDGE) tl = TILE_64x64;
    const int tr = tile_rows(tl), tc = tile_cols(tl);
    const int am = t.M < tr ? t.M : tr, an = t.N < tc ? t.N : tc;
    const double sub = double((am + 15) / 16) * ((an + 15) / 16);
    double c = 64.0;
    for (int i = t.contrib_begin; i < t.contrib_end; ++i) {
      const GContrib& g = cs[i];
      c += (g.flags & GF_IDENT_A) ? 4.0 : g.nred * (((g.K + 3) / 4) * sub + 16.0);
    }
    return c;
  }
  static int64_t jobs_at(const GTask& t, int tl) {
    if (tl == TILE_EDGE) tl = TILE_64x64;
    return (int64_t)((t.M + tile_rows(tl) - 1) / tile_rows(tl)) * ((t.N + tile_cols(tl) - 1) / tile_cols(tl)) *
           t.nbatch;
  }

  // Concatenate host lists, ordering tasks by decreasing job cost so the
  // longest jobs are dispatched first.  Contribution order inside a task is
  // kept, so results do not depend on the ordering.
  static GemmList merge_by_cost(const std::vector<GemmList*>& parts) {
    struct Ref {
      const GemmList* l;
      int t;
      double cost;
    };
    std::vector<Ref> refs;
    GemmList m;
    for (const GemmList* p : parts) {
      for (int t = 0; t < (int)p->tasks.size(); ++t)
        refs.push_back({p, t, job_cost(p->tasks[t], p->contribs.data(), TILE_64x64)});
      m.flops += p->flops;
      m.ngemm += p->ngemm;
      m.reduce.insert(m.reduce.end(), p->reduce.begin(), p->reduce.end());
    }
    std::stable_sort(refs.begin(), refs.end(), [](const Ref& a, const Ref& b) { return a.cost > b.cost; });
    for (const Ref& r : refs) {
      GTask t = r.l->tasks[r.t];
      const int cb = (int)m.contribs.size();
      m.contribs.insert(m.contribs.end(), r.l->contribs.begin() + t.contrib_begin,
                        r.l->contribs.begin() + t.contrib_end);
      t.contrib_begin = cb;
      t.contrib_end = (int)m.contribs.size();
      t.job_begin = m.njobs;
      m.njobs += (int64_t)t.tiles_m * t.tiles_n * t.nbatch;
      m.tasks.push_back(t);
    }
    return m;
  }

  // Task t restricted to rows [m0, m0 + M) and columns [n0, n0 + N) of its
  // output, with tile shape `shape`: the contributions (appended to cx) read
  // their operands from the region's first row and column on.
  static GTask region(const GTask& t, const GContrib* cs, int m0, int n0, int M, int N, int shape,
                      std::vector<GContrib>& cx) {
    GTask g = t;
    g.M = M;
    g.N = N;
    g.shape = shape;
    g.c_off = t.c_off + (int64_t)m0 * t.ldc + n0;
    g.contrib_begin = (int32_t)cx.size();
    for (int i = t.contrib_begin; i < t.contrib_end; ++i) {
      GContrib c = cs[i];
      const bool ta = c.flags & GF_TRANS_A, tb = c.flags & GF_TRANS_B;
      if (c.flags & GF_IDENT_A) {
        c.b_off += tb ? (int64_t)n0 * c.ldb + m0 : (int64_t)m0 * c.ldb + n0;
      } else {
        c.a_off += ta ? (int64_t)m0 : (int64_t)m0 * c.lda;
        c.b_off += tb ? (int64_t)n0 * c.ldb : (int64_t)n0;
      }
      cx.push_back(c);
    }
    g.contrib_end = (int32_t)cx.size();
    return g;
  }

  // Split every task for TILE_EDGE: the interior (rows and columns in whole
  // 64-tiles, plus a last partial 64-tile when more than 32 of it are used)
  // with 64x64 tiles, the rows left over (at most 32) with 32x64 tiles, the
  // columns left over with 64x32 tiles and the corner with 32x32 tiles.  The
  // regions write disjoint parts of C.
  static void split_edges(const std::vector<GTask>& in, const GContrib* cs, std::vector<GTask>& out,
                          std::vector<GContrib>& cx) {
    for (const GTask& t : in) {
      const int rm = t.M % 64, rn = t.N % 64;
      const int Mi = (rm > 0 && rm <= 32) ? t.M - rm : t.M, Ni = (rn > 0 && rn <= 32) ? t.N - rn : t.N;
      const int reg[4][5] = {{0, 0, Mi, Ni, TILE_64x64},
                             {Mi, 0, t.M - Mi, Ni, TILE_32x64},
                             {0, Ni, Mi, t.N - Ni, TILE_64x32},
                             {Mi, Ni, t.M - Mi, t.N - Ni, TILE_32x32}};
      for (const auto& r : reg)
        if (r[2] > 0 && r[3] > 0) out.push_back(region(t, cs, r[0], r[1], r[2], r[3], r[4], cx));
    }
  }

  // Rows (or columns) of a task covered by 128-tiles in TILE_BIG: the whole
  // 128-tiles, plus a last partial one when more than 96 of it are used.
  static int big_extent(int n) { return (n / 128) * 128 + (n % 128 > 96 ? n % 128 : 0); }
  // k tiles (of 32) of one job of task t: its MFMA contributions
  static int64_t k_tiles(const GTask& t, const GContrib* cs) {
    int64_t kt = 0;
    for (int i = t.contrib_begin; i < t.contrib_end; ++i)
      if (!(cs[i].flags & GF_IDENT_A)) kt += (int64_t)cs[i].nred * ((cs[i].K + 31) / 32);
    return kt;
  }
  // TILE_BIG: tasks whose jobs run at least this many k tiles keep their
  // 128-tiled interior in the TILE_128 launch (short k loops stay with the
  // 256-thread shapes, which overlap four workgroups per CU)
  static constexpr int64_t BIG_MIN_KTILES = 32;

  // Count tiles for shape tl, split tasks into job-range pieces, assign them
  // to XCDs (longest processing time first) and upload the per-XCD lists:
  // into fresh device allocations, or into `arena` (nothing is allocated;
  // the lists then live as long as the arena's memory is left alone).
  void upload(int tl, Arena* arena = nullptr, UploadRing* ring = nullptr) {
    DMRG_CHECK(tl >= 0 && tl < NTILE, DMRG_EINVAL, "unknown tile shape");
    free_dev(dev_[tl]);
    if (tl == TILE_BIG) {
      free_dev(rest_);
      big_uploaded_ = false;
    }
    if (tasks.empty()) return;
    if (!reduce.empty() && !dreduce_) {
      DMRG_CHECK(!arena && !ring, DMRG_EINTERNAL, "split-k reduction in an allocation-free list");
      dreduce_ = (ReduceSeg*)dev_alloc_nozero(reduce.size() * sizeof(ReduceSeg));
      dev_h2d(dreduce_, reduce.data(), reduce.size() * sizeof(ReduceSeg));
      nreduce_dev_ = (int)reduce.size();
    }
    // the kernel addresses one k tile of an operand with 32-bit byte offsets
    // from its first element: at most 128 rows (or 32 k) of the leading
    // dimension, which must stay below 2^21 elements
    for (const GContrib& c : contribs)
      DMRG_CHECK(c.lda < (1 << 21) && c.ldb < (1 << 21), DMRG_ESHAPE,
                 "GEMM leading dimension too large for 32-bit tile offsets (limit 2^21 elements)");
    const bool external = arena != nullptr || ring != nullptr;
    // device copy of a host array: a fresh allocation, the arena, or the ring
    auto put = [&](const void* src, size_t b) -> void* {
      if (ring) return ring->stage(src, b);  // one copy for the whole list (flushed below)
      void* p = arena ? arena->take(b) : dev_alloc_nozero(b);
      dev_h2d(p, src, b);
      return p;
    };
    auto own_contribs = [&](Dev& D, const std::vector<GContrib>& cx) {
      D.contribs = (GContrib*)put(cx.data(), cx.size() * sizeof(GContrib));
      D.ncontribs = cx.size();
    };
    if (tl == TILE_EDGE) {
      std::vector<GTask> src;
      std::vector<GContrib> cx;
      split_edges(tasks, contribs.data(), src, cx);
      Dev& D = dev_[tl];
      D.external = external;
      own_contribs(D, cx);
      map_and_put(D, src, cx.data(), put);
    } else if (tl == TILE_BIG) {
      std::vector<GTask> big, rest_in, rest;
      std::vector<GContrib> cbig, crest_in, crest;
      const GContrib* cs = contribs.data();
      for (const GTask& t : tasks) {
        const int Mi = big_extent(t.M), Ni = big_extent(t.N);
        if (Mi > 0 && Ni > 0 && k_tiles(t, cs) >= BIG_MIN_KTILES) {
          big.push_back(region(t, cs, 0, 0, Mi, Ni, TILE_128, cbig));
          if (t.M > Mi) rest_in.push_back(region(t, cs, Mi, 0, t.M - Mi, t.N, TILE_64x64, crest_in));
          if (t.N > Ni) rest_in.push_back(region(t, cs, 0, Ni, Mi, t.N - Ni, TILE_64x64, crest_in));
        } else {
          rest_in.push_back(region(t, cs, 0, 0, t.M, t.N, TILE_64x64, crest_in));
        }
      }
      split_edges(rest_in, crest_in.data(), rest, crest);
      Dev& D = dev_[tl];
      D.external = rest_.external = external;
      if (!big.empty()) {
        own_contribs(D, cbig);
        map_and_put(D, big, cbig.data(), put);
      }
      if (!rest.empty()) {
        own_contribs(rest_, crest);
        map_and_put(rest_, rest, crest.data(), put);
      }
      big_uploaded_ = true;
    } else {
      std::vector<GTask> src = tasks;
      for (GTask& g : src) g.shape = tl;
      Dev& D = dev_[tl];
      D.external = external;
      if (external) {  // own copy of the contributions, in the arena or ring
        own_contribs(D, contribs);
      } else if (!dcontribs_) {
        dcontribs_ = (GContrib*)dev_alloc((contribs.size() + 1) * sizeof(GContrib));
        if (!contribs.empty()) dev_h2d(dcontribs_, contribs.data(), contribs.size() * sizeof(GContrib));
        ncontribs_dev_ = contribs.size();
      }
      map_and_put(D, src, contribs.data(), put);
    }
    if (ring) ring->flush();
  }

  // Split the tasks of one device list (each with its tile shape) into
  // job-range pieces, assign them to XCDs (longest processing time first),
  // and put the per-XCD task lists, bucket table and dynamic units.
  template <class Put>
  static void map_and_put(Dev& D, const std::vector<GTask>& src, const GContrib* cs, Put&& put) {
    std::memset(&D.map, 0, sizeof(D.map));
    std::vector<GTask> dev;
    std::vector<double> cj(src.size());
    std::vector<int64_t> nj(src.size());
    double total = 0;
    for (size_t t = 0; t < src.size(); ++t) {
      cj[t] = job_cost(src[t], cs, src[t].shape);
      nj[t] = jobs_at(src[t], src[t].shape);
      total += cj[t] * nj[t];
    }
    const double piece_cost = std::max(total / (NXCD * 32.0), 1.0);
    struct Piece {
      size_t t;
      int64_t off, n;
      double c;
    };
    std::vector<Piece> pcs;
    for (size_t t = 0; t < src.size(); ++t) {
      int64_t np = (int64_t)std::ceil(cj[t] * nj[t] / piece_cost);
      np = std::max<int64_t>(1, std::min<int64_t>(np, nj[t]));
      for (int64_t i = 0; i < np; ++i) {
        const int64_t a = nj[t] * i / np, b = nj[t] * (i + 1) / np;
        if (b > a) pcs.push_back({t, a, b - a, cj[t]});
      }
    }
    std::stable_sort(pcs.begin(), pcs.end(), [](const Piece& a, const Piece& b) { return a.c * a.n > b.c * b.n; });
    std::vector<std::vector<Piece>> per(NXCD);
    double load[NXCD] = {0};
    for (const Piece& p : pcs) {
      int x = 0;
      for (int i = 1; i < NXCD; ++i)
        if (load[i] < load[x]) x = i;
      load[x] += p.c * p.n;
      per[x].push_back(p);
    }
    // Units for dynamic launches (guided self-scheduling): a unit of
    // consecutive jobs takes about 1/(4 S) of the work left on its XCD, with
    // S the workgroups resident per XCD (128 of the 256-thread shapes, 32 of
    // TILE_128), and at least one job.
    const double S = (!src.empty() && src[0].shape == TILE_128) ? 32.0 : 128.0;
    std::vector<int64_t> units;
    for (int x = 0; x < NXCD; ++x) {
      // longest jobs first inside an XCD
      std::stable_sort(per[x].begin(), per[x].end(), [](const Piece& a, const Piece& b) { return a.c > b.c; });
      D.map.task_begin[x] = (int)dev.size();
      D.map.unit_begin[x] = (int64_t)units.size();
      double rem = load[x];
      int64_t jb = 0;
      for (const Piece& p : per[x]) {
        for (int64_t left = p.n, j = jb; left > 0;) {
          const double target = std::max(p.c, rem / (4.0 * S));
          const int64_t g = std::max<int64_t>(1, std::min<int64_t>(left, (int64_t)(target / p.c)));
          units.push_back(j);
          j += g;
          left -= g;
          rem -= p.c * g;
        }
        GTask g = src[p.t];
        g.tiles_m = (g.M + tile_rows(g.shape) - 1) / tile_rows(g.shape);
        g.tiles_n = (g.N + tile_cols(g.shape) - 1) / tile_cols(g.shape);
        g.job_begin = jb;
        g.job_off = p.off;
        g.njob = p.n;
        jb += p.n;
        dev.push_back(g);
      }
      D.map.njobs[x] = jb;
      D.map.max_jobs = std::max(D.map.max_jobs, jb);
      units.push_back(jb);
      D.map.nunits[x] = (int64_t)units.size() - 1 - D.map.unit_begin[x];
    }
    D.units = (int64_t*)put(units.data(), units.size() * sizeof(int64_t));
    const std::vector<unsigned> zeros(64 * NXCD, 0u);
    D.counters = (unsigned*)put(zeros.data(), zeros.size() * sizeof(unsigned));
    D.map.units = D.units;
    D.map.counters = D.counters;
    D.map.task_begin[NXCD] = (int)dev.size();
    D.map.shift = 0;
    while ((D.map.max_jobs >> D.map.shift) > (int64_t(1) << 14)) ++D.map.shift;
    std::vector<int> bucket;
    for (int x = 0; x < NXCD; ++x) {
      D.map.bucket_begin[x] = (int)bucket.size();
      const int tb = D.map.task_begin[x], te = D.map.task_begin[x + 1];
      const int64_t nb = (D.map.njobs[x] >> D.map.shift) + 1;
      int ti = tb;
      for (int64_t b = 0; b <= nb; ++b) {
        const int64_t job = b << D.map.shift;
        while (ti + 1 < te && dev[ti + 1].job_begin <= job) ++ti;
        bucket.push_back(te > tb ? ti : tb);
      }
    }
    D.map.bucket_begin[NXCD] = (int)bucket.size();
    D.bucket = (int*)put(bucket.data(), bucket.size() * sizeof(int));
    D.tasks = (GTask*)put(dev.data(), dev.size() * sizeof(GTask));
    D.ntasks = (int)dev.size();
  }
  void upload() { upload(tile); }
  bool uploaded(int tl) const {
    return tasks.empty() || (tl == TILE_BIG ? big_uploaded_ : dev_[tl].tasks != nullptr);
  }
  void run(DevTable& tab, const void* p0, void* p1, int elem, void* stream) { run_tile(tile, tab, p0, p1, elem, stream); }
  void run_tile(int tl, DevTable& tab, const void* p0, void* p1, int elem, void* stream) {
    if (!uploaded(tl)) upload(tl);
    run_uploaded(tl, tab.device(), p0, p1, elem, stream);
  }
  // launch the lists uploaded for shape tl with a device pointer table
  void run_uploaded(int tl, void* const* table_dev, const void* p0, void* p1, int elem, void* stream) {
    auto launch = [&](const Dev& D, int shape) {
      if (D.ntasks == 0) return;
      gemm_launch(D.tasks, D.ntasks, D.map, D.contribs ? D.contribs : dcontribs_, D.bucket, table_dev, p0, p1, elem,
                  shape, grid_per_xcd, stream);
    };
    if (tl == TILE_BIG) {  // the 128x128 interiors, then everything else
      launch(dev_[TILE_BIG], TILE_128);
      launch(rest_, TILE_EDGE);
    } else {
      launch(dev_[tl], tl);
    }
    if (nreduce_dev_) reduce_launch(dreduce_, nreduce_dev_, table_dev, p1, stream);
  }
  void release() {
    for (int t = 0; t < NTILE; ++t) free_dev(dev_[t]);
    free_dev(rest_);
    big_uploaded_ = false;
    dev_free(dreduce_);
    dreduce_ = nullptr;
    nreduce_dev_ = 0;
    dev_free(dcontribs_);
    dcontribs_ = nullptr;
    ncontribs_dev_ = 0;
  }
  // drop the device copy of one tile shape (rebuilt on demand from the host list)
  void release_tile(int t) {
    if (tasks.empty()) return;
    free_dev(dev_[t]);
    if (t == TILE_BIG) {
      free_dev(rest_);
      big_uploaded_ = false;
    }
  }
  void clear_host() {
    std::vector<GTask>().swap(tasks);
    std::vector<GContrib>().swap(contribs);
    std::vector<ReduceSeg>().swap(reduce);
  }
  size_t host_bytes() const { return tasks.size() * sizeof(GTask) + contribs.size() * sizeof(GContrib); }
  size_t device_bytes() const {
    size_t b = ncontribs_dev_ * sizeof(GContrib);
    for (int t = 0; t < NTILE; ++t) b += (size_t)dev_[t].ntasks * sizeof(GTask) + dev_[t].ncontribs * sizeof(GContrib);
    b += (size_t)rest_.ntasks * sizeof(GTask) + rest_.ncontribs * sizeof(GContrib);
    return b;
  }

 private:
  struct Dev {
    GTask* tasks = nullptr;
    int* bucket = nullptr;
    GContrib* contribs = nullptr;  // own contribution array (TILE_EDGE), else the shared one
    int64_t* units = nullptr;      // unit boundaries of dynamic launches
    unsigned* counters = nullptr;  // per-XCD unit counters of dynamic launches
    size_t ncontribs = 0;
    XcdMap map{};
    int ntasks = 0;
    bool external = false;         // placed in an Arena: not freed here
  };
  static void free_dev(Dev& d) {
    if (d.external) {
      d = Dev{};
      return;
    }
    dev_free(d.tasks);
    dev_free(d.bucket);
    dev_free(d.contribs);
    dev_free(d.units);
    dev_free(d.counters);
    d = Dev{};
  }
  bool any_dev() const {
    for (int t = 0; t < NTILE; ++t)
      if (dev_[t].ntasks) return true;
    return rest_.ntasks != 0;
  }
  GContrib* dcontribs_ = nullptr;
  size_t ncontribs_dev_ = 0;
  Dev dev_[NTILE];
  Dev rest_;                  // TILE_BIG: the launch after the 128x128 interiors
  bool big_uploaded_ = false;
  ReduceSeg* dreduce_ = nullptr;
  int nreduce_dev_ = 0;
};

inline GContrib make_contrib(int K, int flags, int a_buf, int64_t a_off, int lda, int b_buf, int64_t b_off,
                             int ldb, double alpha) {
  GContrib c{};
  c.K = K;
  c.flags = flags;
  c.a_buf = a_buf;
  c.b_buf = b_buf;
  c.s_buf = -1;
  c.lda = lda;
  c.ldb = ldb;
  c.nred = 1;
  c.alpha = alpha;
  c.a_off = a_off;
  c.b_off = b_off;
  return c;
}

}  // namespace dmrg
