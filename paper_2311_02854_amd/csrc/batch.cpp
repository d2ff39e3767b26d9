// sigma for many independent problems in one fused launch sequence.
//
// Launch j of the fused sequence holds launch j of every problem (each
// problem's own sequence is [L(id) + R(0)], [L(0) + R(1)], ..., so the
// dependences between its launches are kept), with every problem's buffer ids
// moved into one pointer table.  Tiles of all problems share the XCD
// schedule, so small problems fill the tails of large ones.  The sequence
// (sigma clears, FP32 conversions of psi, GEMM launches) is captured once
// into an executable HIP graph and replayed while the psi/sigma pointers stay
// the same; launch shapes come from the autotuner.
#include <cstring>

#include "batch.h"

namespace dmrg {

namespace {
int remap(int id, int base, int psi_id, int sig_id) {
  if (id < 0) return id;
  if (id == 0) return psi_id;
  if (id == 1) return sig_id;
  return base + id - 2;
}
}  // namespace

BatchPlan::~BatchPlan() {
  graph_destroy(graph);
  stream_destroy(cap_stream);
  for (void* e : events) ev_destroy(e);
}

bool BatchPlan::matches(const std::vector<Ops*>& ops, int p) const {
  if (p != prec || ops.size() != probs.size()) return false;
  for (size_t i = 0; i < ops.size(); ++i)
    if (ops[i] != probs[i] || ops[i]->serial != serials[i]) return false;
  return true;
}

std::unique_ptr<BatchPlan> build_batch(const std::vector<Ops*>& ops, int prec, void* stream) {
  DMRG_CHECK(!ops.empty(), DMRG_EINVAL, "no problems");
  auto B = std::make_unique<BatchPlan>();
  B->probs = ops;
  B->prec = prec;
  for (Ops* O : ops) {
    B->serials.push_back(O->serial);
    if (prec != P_F64) make_reduced_copies(*O, stream);
  }
  B->tab = std::make_unique<DevTable>();
  DevTable& tab = *B->tab;
  std::vector<int> base(ops.size());
  size_t nl = 0;
  for (size_t p = 0; p < ops.size(); ++p) {
    const Ops& O = *ops[p];
    const DevTable& src = prec == P_F64 ? *O.tab : *O.tab32;
    base[p] = tab.size();
    for (int id = 2; id < src.size(); ++id) tab.add(src.get(id));
    B->psi_id.push_back(tab.add(nullptr));
    B->sig_id.push_back(tab.add(nullptr));
    nl = std::max(nl, O.launches.size());
    for (const GemmList& l : O.launches)
      DMRG_CHECK(!l.tasks.empty(), DMRG_EINTERNAL, "a sigma launch has no host task list");
  }
  for (size_t j = 0; j < nl; ++j) {
    std::vector<GemmList> parts;
    for (size_t p = 0; p < ops.size(); ++p) {
      const Ops& O = *ops[p];
      if (j >= O.launches.size()) continue;
      const GemmList& src = O.launches[j];
      GemmList g;
      g.tasks = src.tasks;
      g.contribs = src.contribs;
      g.flops = src.flops;
      g.ngemm = src.ngemm;
      const int b = base[p], pi = B->psi_id[p], si = B->sig_id[p];
      for (GTask& t : g.tasks) t.c_buf = remap(t.c_buf, b, pi, si);
      for (GContrib& c : g.contribs) {
        c.a_buf = (c.flags & GF_IDENT_A) ? c.a_buf : remap(c.a_buf, b, pi, si);
        c.b_buf = remap(c.b_buf, b, pi, si);
        c.s_buf = remap(c.s_buf, b, pi, si);
      }
      g.reduce = src.reduce;
      for (ReduceSeg& r : g.reduce) {
        r.dst_buf = remap(r.dst_buf, b, pi, si);
        r.src_buf = remap(r.src_buf, b, pi, si);
      }
      parts.push_back(std::move(g));
    }
    std::vector<GemmList*> pp;
    for (auto& g : parts) pp.push_back(&g);
    GemmList m = GemmList::merge_by_cost(pp);
    m.upload(TILE_64x64);
    B->flops += m.flops;
    B->launches.push_back(std::move(m));
  }
  B->tiles.assign(B->launches.size(), TILE_64x64);
  B->grids.assign(B->launches.size(), 0);
  B->psi_cur.assign(ops.size(), nullptr);
  B->sig_cur.assign(ops.size(), nullptr);
  return B;
}

void BatchPlan::bind(const double* const* psi, double* const* sigma, void* stream) {
  bool changed = false;
  for (size_t p = 0; p < probs.size(); ++p)
    changed |= psi_cur[p] != psi[p] || sig_cur[p] != sigma[p];
  if (!changed) return;
  dev_sync(stream);  // launches in flight may still read the table
  for (size_t p = 0; p < probs.size(); ++p) {
    psi_cur[p] = psi[p];
    sig_cur[p] = sigma[p];
    tab->set(psi_id[p], prec == P_F64 ? (void*)psi[p] : (void*)probs[p]->psi32);
    tab->set(sig_id[p], sigma[p]);
  }
  tab->device();
  graph_destroy(graph);
  graph = nullptr;
}

void BatchPlan::issue(void* s, const std::vector<int>& tl, const std::vector<int64_t>& gr,
                      std::vector<double>* ms) {
  for (size_t p = 0; p < probs.size(); ++p) {
    k_fill(sig_cur[p], 0.0, probs[p]->npsi, s);
    if (prec != P_F64) k_d2f(psi_cur[p], probs[p]->psi32, probs[p]->npsi, s);
    gather_psi(*probs[p], psi_cur[p], prec, s);
  }
  if (ms) {
    while (events.size() < launches.size() + 1) events.push_back(ev_create());
    ev_record(events[0], s);
  }
  for (size_t j = 0; j < launches.size(); ++j) {
    launches[j].grid_per_xcd = gr[j];
    launches[j].run_tile(tl[j], *tab, nullptr, nullptr, prec, s);
    if (ms) ev_record(events[j + 1], s);
  }
  if (ms)
    for (size_t j = 0; j < launches.size(); ++j) (*ms)[j] = ev_elapsed_ms(events[j], events[j + 1]);
}

void BatchPlan::autotune(void* stream) {
  auto run_all = [&](const std::vector<int>& tl, const std::vector<int64_t>& gr, std::vector<double>& ms) {
    issue(stream, tl, gr, &ms);
  };
  autotune_launches(launches.size(), run_all, tiles, grids, ms_default, ms_best);
  for (size_t j = 0; j < launches.size(); ++j)
    for (int t = 0; t < NTILE; ++t)
      if (t != tiles[j]) launches[j].release_tile(t);
  tuned = true;
  graph_destroy(graph);
  graph = nullptr;
}

void BatchPlan::run(const double* const* psi, double* const* sigma, bool use_graph, void* stream) {
  bind(psi, sigma, stream);
  if (!use_graph) {
    issue(stream, tiles, grids, nullptr);
    return;
  }
  if (!graph) {
    // everything the captured work reads must already be on the device
    for (size_t j = 0; j < launches.size(); ++j)
      if (!launches[j].uploaded(tiles[j])) launches[j].upload(tiles[j]);
    tab->device();
    if (!cap_stream) cap_stream = stream_create();
    graph_begin(cap_stream);
    try {
      issue(cap_stream, tiles, grids, nullptr);
    } catch (...) {
      try {
        graph_destroy(graph_end(cap_stream));
      } catch (...) {
      }
      throw;
    }
    graph = graph_end(cap_stream);
  }
  graph_launch(graph, stream);
}

}  // namespace dmrg
