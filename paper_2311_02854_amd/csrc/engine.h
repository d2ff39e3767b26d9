// Host-side helpers around the grouped GEMM kernel: a device pointer table
// and a task-list builder.
#pragma once
#include <memory>
#include <vector>

#include "common.h"
#include "device.h"

namespace dmrg {

// Table of device pointers addressed by buffer id (ids 0 and 1 are the
// per-launch pointers p0 / p1 of gemm_launch).
class DevTable {
 public:
  DevTable() : ptrs_{nullptr, nullptr} {}
  ~DevTable() { dev_free(dev_); }
  DevTable(const DevTable&) = delete;
  DevTable& operator=(const DevTable&) = delete;
  int add(void* p) {
    ptrs_.push_back(p);
    dirty_ = true;
    return (int)ptrs_.size() - 1;
  }
  void set(int id, void* p) {
    ptrs_[id] = p;
    dirty_ = true;
  }
  void* get(int id) const { return ptrs_[id]; }
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

 private:
  std::vector<void*> ptrs_;
  void** dev_ = nullptr;
  size_t cap_ = 0;
  bool dirty_ = true;
};

// A list of GEMM tasks executed by one gemm_launch.
class GemmList {
 public:
  static constexpr int TILE = 64;
  std::vector<GTask> tasks;
  std::vector<GContrib> contribs;
  int64_t njobs = 0;
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
      tasks = std::move(o.tasks);
      contribs = std::move(o.contribs);
      njobs = o.njobs;
      flops = o.flops;
      ngemm = o.ngemm;
      dtasks_ = o.dtasks_;
      dcontribs_ = o.dcontribs_;
      dbucket_ = o.dbucket_;
      shift_ = o.shift_;
      ntasks_dev_ = o.ntasks_dev_;
      o.dtasks_ = nullptr;
      o.dcontribs_ = nullptr;
      o.dbucket_ = nullptr;
    }
    return *this;
  }

  void begin(int M, int N, int nbatch, int c_buf, int64_t c_off, int ldc, int64_t c_bstride, bool accumulate) {
    GTask t{};
    t.M = M;
    t.N = N;
    t.nbatch = nbatch;
    t.tiles_m = (M + TILE - 1) / TILE;
    t.tiles_n = (N + TILE - 1) / TILE;
    t.c_buf = c_buf;
    t.ldc = ldc;
    t.accumulate = accumulate ? 1 : 0;
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
        (t.contrib_begin == t.contrib_end && t.accumulate)) {
      contribs.resize(t.contrib_begin);
      tasks.pop_back();
      return;
    }
    t.job_begin = njobs;
    njobs += (int64_t)t.tiles_m * t.tiles_n * t.nbatch;
  }
  bool empty() const { return tasks.empty() && ntasks_dev_ == 0; }
  void upload() {
    release();
    ntasks_dev_ = (int)tasks.size();
    if (tasks.empty()) return;
    dtasks_ = (GTask*)dev_alloc(tasks.size() * sizeof(GTask));
    dev_h2d(dtasks_, tasks.data(), tasks.size() * sizeof(GTask));
    dcontribs_ = (GContrib*)dev_alloc((contribs.size() + 1) * sizeof(GContrib));
    if (!contribs.empty()) dev_h2d(dcontribs_, contribs.data(), contribs.size() * sizeof(GContrib));
    // bucket table: at most 2^16 buckets of 2^shift jobs
    shift_ = 0;
    while ((njobs >> shift_) > (int64_t(1) << 16)) ++shift_;
    const int64_t nb = (njobs >> shift_) + 1;
    std::vector<int> bucket((size_t)nb + 1);
    size_t ti = 0;
    for (int64_t b = 0; b <= nb; ++b) {
      const int64_t job = b << shift_;
      while (ti + 1 < tasks.size() && tasks[ti + 1].job_begin <= job) ++ti;
      bucket[(size_t)b] = (int)ti;
    }
    dbucket_ = (int*)dev_alloc(bucket.size() * sizeof(int));
    dev_h2d(dbucket_, bucket.data(), bucket.size() * sizeof(int));
  }
  void run(DevTable& tab, const void* p0, void* p1, int elem, void* stream) {
    if (!dtasks_) upload();
    if (ntasks_dev_ == 0) return;
    gemm_launch(dtasks_, ntasks_dev_, njobs, dcontribs_, dbucket_, shift_, tab.device(), p0, p1, elem, stream);
  }
  void release() {
    dev_free(dtasks_);
    dev_free(dcontribs_);
    dev_free(dbucket_);
    dtasks_ = nullptr;
    dcontribs_ = nullptr;
    dbucket_ = nullptr;
  }
  void clear_host() {
    std::vector<GTask>().swap(tasks);
    std::vector<GContrib>().swap(contribs);
  }

 private:
  GTask* dtasks_ = nullptr;
  GContrib* dcontribs_ = nullptr;
  int* dbucket_ = nullptr;
  int shift_ = 0;
  int ntasks_dev_ = 0;
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
