// Fused multi-problem sigma plan (see batch.cpp).
#pragma once
#include <memory>
#include <vector>

#include "ops.h"

namespace dmrg {

struct BatchPlan {
  std::vector<Ops*> probs;
  std::vector<uint64_t> serials;
  int prec = P_F64;
  std::unique_ptr<DevTable> tab;        // every problem's buffers, one id space
  std::vector<int> psi_id, sig_id;      // table ids of each problem's psi / sigma
  std::vector<GemmList> launches;       // fused launch j = launch j of every problem
  std::vector<int> tiles;               // launch shapes (autotuned)
  std::vector<int64_t> grids;
  bool tuned = false;
  double flops = 0, ms_default = 0, ms_best = 0;
  std::vector<const double*> psi_cur;   // pointers the table holds
  std::vector<double*> sig_cur;
  void* graph = nullptr;                // executable graph of the whole sequence
  void* cap_stream = nullptr;
  std::vector<void*> events;

  ~BatchPlan();
  bool matches(const std::vector<Ops*>& ops, int prec) const;
  void bind(const double* const* psi, double* const* sigma, void* stream);
  void issue(void* s, const std::vector<int>& tiles, const std::vector<int64_t>& grids, std::vector<double>* ms);
  void autotune(void* stream);
  void run(const double* const* psi, double* const* sigma, bool use_graph, void* stream);
};

std::unique_ptr<BatchPlan> build_batch(const std::vector<Ops*>& ops, int prec, void* stream);

}  // namespace dmrg
