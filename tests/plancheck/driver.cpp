// Plan bounds checker driver (test infrastructure only).
//
// Reads one two-dot problem written by tests/test_plan_bounds.py, builds its
// operators through the C ABI on the dry-run device layer (stub_device.cpp),
// then issues sigma in every precision with every launch shape (each tile
// shape, one workgroup per job and dynamic units), diag(H) and,
// with a second copy of the problem, the fused two-problem sigma.  The
// device layer checks every launch's addressing; this program only drives it.
//
//   plancheck INPUT X_BUDGET_BYTES full|short [batched|noalloc_fails]
// full: sigma with every launch shape, one workgroup per job and dynamic units
// (a persistent grid only strides the same jobs); short: the 64x64, mixed and
// big shapes only (the other shapes share their addressing code); batched: also
// the fused two-problem sigma; noalloc_fails:
// dmrg_diag_noalloc must refuse (run with a static scratch set too small)
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dmrg.h"
#include "../../paper_2311_02854_amd/csrc/common.h"
#include "../../paper_2311_02854_amd/csrc/device.h"

namespace dmrg {
void plancheck_report();
int64_t plancheck_alloc_count();
}

template <typename T>
static std::vector<T> rd(FILE* f, size_t n) {
  std::vector<T> v(n);
  if (n && std::fread(v.data(), sizeof(T), n, f) != n) {
    std::fprintf(stderr, "short input\n");
    std::exit(2);
  }
  return v;
}

static void ok(int rc, dmrg_ctx* ctx, const char* what) {
  if (rc != 0) {
    std::fprintf(stderr, "%s failed (%d): %s\n", what, rc, dmrg_last_error(ctx));
    std::exit(1);
  }
}

// The checker itself: a task whose operand tile reaches one element past its
// buffer, and one whose leading dimension overflows the 32-bit tile offsets,
// must both be refused.
static int selftest() {
  using namespace dmrg;
  int refused = 0;
  for (int variant = 0; variant < 2; ++variant) {
    const int M = 64, N = 64, K = 40;
    const int lda = variant == 0 ? K : (1 << 23);
    const size_t na = variant == 0 ? (size_t)M * K - 1 : (size_t)M * lda;   // one element short
    double* A = (double*)dev_alloc(na * 8);
    double* B = (double*)dev_alloc((size_t)K * N * 8);
    double* Cm = (double*)dev_alloc((size_t)M * N * 8);
    void* tab_h[4] = {nullptr, nullptr, A, B};
    void** tab = (void**)dev_alloc(sizeof tab_h);
    dev_h2d(tab, tab_h, sizeof tab_h);
    GContrib c{};
    c.K = K;
    c.a_buf = 2;
    c.b_buf = 3;
    c.s_buf = -1;
    c.lda = lda;
    c.ldb = N;
    c.nred = 1;
    c.alpha = 1.0;
    GContrib* dc = (GContrib*)dev_alloc(sizeof c);
    dev_h2d(dc, &c, sizeof c);
    GTask t{};
    t.M = M;
    t.N = N;
    t.nbatch = 1;
    t.tiles_m = t.tiles_n = 1;
    t.c_buf = 1;
    t.ldc = N;
    t.accumulate = GT_C64;
    t.contrib_begin = 0;
    t.contrib_end = 1;
    t.njob = 1;
    GTask* dt = (GTask*)dev_alloc(sizeof t);
    dev_h2d(dt, &t, sizeof t);
    XcdMap map{};
    map.task_begin[1] = map.task_begin[NXCD] = 1;
    for (int x = 1; x < NXCD; ++x) map.task_begin[x] = 1;
    map.njobs[0] = map.max_jobs = 1;
    int bk_h[3] = {0, 0, 0};
    int* bk = (int*)dev_alloc(sizeof bk_h);
    dev_h2d(bk, bk_h, sizeof bk_h);
    try {
      gemm_launch(dt, 1, map, dc, bk, tab, nullptr, Cm, P_F64, TILE_64x64, 0, nullptr);
      std::printf("selftest variant %d was not refused\n", variant);
    } catch (const Error& e) {
      std::printf("selftest variant %d refused: %s\n", variant, e.what());
      const char* want = variant == 0 ? "outside the allocation" : "exceed 32 bits";
      if (std::strstr(e.what(), want)) ++refused;
    }
    for (void* p : {(void*)A, (void*)B, (void*)Cm, (void*)tab, (void*)dc, (void*)dt, (void*)bk}) dev_free(p);
  }
  return refused == 2 ? 0 : 1;
}

int main(int argc, char** argv) {
  if (argc == 2 && std::string(argv[1]) == "selftest") return selftest();
  if (argc < 3) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  const size_t x_budget = std::strtoull(argv[2], nullptr, 10);
  const bool quick = argc > 3 && std::string(argv[3]) == "short";
  const bool batched = argc > 4 && std::string(argv[4]) == "batched";
  const bool expect_noalloc_fail = argc > 4 && std::string(argv[4]) == "noalloc_fails";
  auto hdr = rd<int64_t>(f, 6);  // K, Na, Nb, bond, total sectors, blocks
  const int K = (int)hdr[0];
  auto nsec = rd<int>(f, (size_t)K + 1);
  auto sec_qn = rd<int>(f, 2 * (size_t)hdr[4]);
  auto sec_dim = rd<int>(f, (size_t)hdr[4]);
  auto blk_off = rd<int64_t>(f, (size_t)hdr[5]);
  auto ndata = rd<int64_t>(f, 1);
  auto data = rd<double>(f, (size_t)ndata[0]);
  auto h = rd<double>(f, (size_t)K * K);
  auto eri = rd<double>(f, (size_t)K * K * K * K);
  std::fclose(f);

  dmrg_ctx* ctx = nullptr;
  ok(dmrg_create(&ctx, 0, nullptr), ctx, "create");
  dmrg_integrals I{K, h.data(), eri.data(), 0.0};
  dmrg_mps M{K, (int)hdr[1], (int)hdr[2], (int)hdr[3], nsec.data(), sec_qn.data(), sec_dim.data(),
             blk_off.data(), data.data()};
  // PLANCHECK_KSPLIT: split-k threshold of sigma's L-step (default when unset)
  const char* ks = std::getenv("PLANCHECK_KSPLIT");
  dmrg_build_opts bo{x_budget, 0, ks ? std::atoll(ks) : 0};
  dmrg_ops* ops = nullptr;
  ok(dmrg_build_ops(ctx, &I, &M, &bo, &ops), ctx, "build_ops");
  int64_t npsi = 0, nb = 0;
  ok(dmrg_ops_layout(ops, &npsi, &nb, nullptr, nullptr), ctx, "layout");
  double* psi = (double*)dmrg::dev_alloc(sizeof(double) * (size_t)npsi);
  double* sig = (double*)dmrg::dev_alloc(sizeof(double) * (size_t)npsi);
  for (int prec = 0; prec < 3; ++prec)
    for (int tile = 0; tile < dmrg::NTILE; ++tile)
      for (int64_t grid : {int64_t(0), int64_t(-1)}) {
        if (quick && tile != dmrg::TILE_64x64 && tile != dmrg::TILE_EDGE && tile != dmrg::TILE_BIG)
          continue;
        ok(dmrg_launch_shape(ops, prec, tile, grid), ctx, "launch_shape");
        ok(dmrg_sigma(ctx, ops, psi, sig, prec), ctx, "sigma");
      }
  ok(dmrg_diag(ctx, ops, sig), ctx, "diag");
  {
    // the allocation-free diag: no dev_alloc at all, every launch checked
    const int64_t before = dmrg::plancheck_alloc_count();
    const int rc = dmrg_diag_noalloc(ctx, ops, sig);
    if (expect_noalloc_fail) {
      if (rc != DMRG_ENOMEM) {
        std::fprintf(stderr, "diag_noalloc with a small scratch returned %d, not DMRG_ENOMEM\n", rc);
        return 1;
      }
      std::printf("diag_noalloc refused: %s\n", dmrg_last_error(ctx));
    } else {
      ok(rc, ctx, "diag_noalloc");
    }
    if (dmrg::plancheck_alloc_count() != before) {
      std::fprintf(stderr, "diag_noalloc allocated device memory\n");
      return 1;
    }
  }
  if (batched) {
    dmrg_ops* ops2 = nullptr;
    ok(dmrg_build_ops(ctx, &I, &M, &bo, &ops2), ctx, "build_ops (second)");
    double* psi2 = (double*)dmrg::dev_alloc(sizeof(double) * (size_t)npsi);
    double* sig2 = (double*)dmrg::dev_alloc(sizeof(double) * (size_t)npsi);
    dmrg_ops* const list[2] = {ops, ops2};
    const double* const ps[2] = {psi, psi2};
    double* const ss[2] = {sig, sig2};
    for (int prec = 0; prec < 3; ++prec)
      for (int flags : {0, DMRG_BATCH_EAGER | DMRG_BATCH_NO_TUNE})
        ok(dmrg_sigma_batched(ctx, 2, list, ps, ss, prec, flags), ctx, "sigma_batched");
    dmrg_ops_destroy(ops2);
    dmrg::dev_free(psi2);
    dmrg::dev_free(sig2);
  }
  dmrg_stats st;
  ok(dmrg_ops_stats(ops, &st), ctx, "stats");
  std::printf("n_psi %lld blocks %lld sigma %.4f TFLOP build %.4f TFLOP\n", (long long)npsi, (long long)nb,
              st.flops_sigma / 1e12, st.build_flops / 1e12);
  dmrg_ops_destroy(ops);
  dmrg::dev_free(psi);
  dmrg::dev_free(sig);
  dmrg_destroy(ctx);
  dmrg::plancheck_report();
  std::printf("PLANCHECK OK\n");
  return 0;
}
