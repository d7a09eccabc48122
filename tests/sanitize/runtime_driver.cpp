// Calls the host-side entry points of libimloc (argument checks, planning,
// workspace and staging sizes, paper settings) for a build of the runtime
// with AddressSanitizer and UndefinedBehaviorSanitizer on its host code (test
// infrastructure: tests/test_sanitizers.py builds and runs it on a machine
// without a GPU, where context creation must fail cleanly).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "imloc.h"

int main() {
  int fails = 0;
  auto check = [&](bool ok, const char* what) {
    if (!ok) {
      std::fprintf(stderr, "failed: %s\n", what);
      ++fails;
    }
  };
  imloc_ransac_params p;
  check(imloc_paper_params(6.0, &p) == IMLOC_OK, "paper params");
  check(imloc_paper_params(NAN, &p) == IMLOC_EINVAL, "paper params NaN");
  check(imloc_paper_params(4.0, nullptr) == IMLOC_EINVAL, "paper params null");
  p.fixed_samples = 4096;
  p.batch = 4096;
  const size_t one = imloc_workspace_bytes(50000, &p);
  check(one > 0, "workspace bytes");
  // batches of 1 to 40 queries: the host plan's containers grow past their inline room
  for (int nq : {1, 3, 4, 5, 17, 40}) {
    std::vector<int64_t> n(nq);
    for (int q = 0; q < nq; ++q) n[q] = 1000 + 997 * q;
    std::vector<imloc_ransac_params> ps(nq, p);
    for (int q = 0; q < nq; ++q) ps[q].lo_top_k = 1 + q % 9;
    const size_t b1 = imloc_batch_workspace_bytes(nq, n.data(), &p, 1);
    const size_t b2 = imloc_batch_workspace_bytes(nq, n.data(), ps.data(), nq);
    check(b1 > 0 && b2 > 0, "batch workspace bytes");
    check(imloc_staging_bytes(nq, nq) >= (size_t)nq * 700, "staging bytes");
    std::vector<int32_t> nc(nq, 2);
    (void)nc;
  }
  imloc_rig_camera cams[2];
  std::memset(cams, 0, sizeof(cams));
  check(imloc_rig_workspace_bytes(20000, 4, &p) > 0, "rig workspace bytes");
  check(imloc_score_workspace_bytes(1000, 64, 0) > 0, "score workspace bytes");
  check(imloc_lift_workspace_bytes(160000, 20) > 0, "lift workspace bytes");
  check(imloc_lo_workspace_bytes(5000, 8) > 0, "lo workspace bytes");
  check(imloc_refine_workspace_bytes(5000) > 0, "refine workspace bytes");
  check(imloc_sample_workspace_bytes(2000, 1024) > 0, "sample workspace bytes");
  check(imloc_triangulate_workspace_bytes(560, 560, 10) > 0, "triangulate workspace bytes");
  check(imloc_rig_stage_workspace_bytes(2000, 2, 100) > 0, "rig stage workspace bytes");
  check(imloc_noalloc_max_bytes() == (size_t(32) << 20), "noalloc size");
  imloc_server_config cfg{64, 8, 200000, 64 * 4096, 64 * 200256};
  check(imloc_server_workspace_bytes(&cfg) > 0, "server workspace bytes");
  cfg.max_slots = 0;
  check(imloc_server_workspace_bytes(&cfg) == 0, "bad server config");
  // calls without a context
  imloc_pose pose;
  check(imloc_lo_ransac_pnp(nullptr, nullptr, 0, nullptr, &p, &pose, nullptr, nullptr) == IMLOC_EINVAL, "null ctx");
  check(imloc_lo_ransac_pnp_noalloc(nullptr, nullptr, 0, nullptr, &p, &pose, nullptr, nullptr) == IMLOC_EINVAL,
        "null ctx noalloc");
  check(imloc_set_workspace(nullptr, nullptr, 0) == IMLOC_EINVAL, "null ctx workspace");
  check(imloc_set_staging(nullptr, 4096) == IMLOC_EINVAL, "null ctx staging");
  check(imloc_get_staging(nullptr) == 0, "null ctx get staging");
  int32_t pts = 0;
  check(imloc_set_score_points(nullptr, 2048) == IMLOC_EINVAL, "null ctx score points");
  check(imloc_get_score_points(nullptr, &pts) == IMLOC_EINVAL, "null ctx get score points");
  check(std::strcmp(imloc_last_error(nullptr), "null context") == 0, "null ctx error");
  // no GPU here: creating a context fails cleanly
  imloc_ctx* ctx = nullptr;
  const int rc = imloc_create(&ctx, 0, nullptr);
  check(rc != IMLOC_OK && ctx == nullptr, "create without a device");
  std::printf("runtime driver done: %d failure(s)\n", fails);
  return fails ? 1 : 0;
}
