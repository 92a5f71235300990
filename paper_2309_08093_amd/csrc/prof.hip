// Opt-in per-kernel-class timing with HIP events on the plan's stream.
#include <utility>
#include <vector>

#include "tt_internal.h"

namespace {
struct ProfState {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> done[TT_PROF_NCLASS];
  hipEvent_t open[TT_PROF_NCLASS] = {};
};
}  // namespace

void tt_prof_begin(const tt_plan_s* p, int cls) {
  if (!p->prof) return;
  ProfState* st = static_cast<ProfState*>(p->prof);
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  hipEventRecord(e, p->stream);
  st->open[cls] = e;
}

void tt_prof_end(const tt_plan_s* p, int cls) {
  if (!p->prof) return;
  ProfState* st = static_cast<ProfState*>(p->prof);
  if (!st->open[cls]) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  hipEventRecord(e, p->stream);
  st->done[cls].emplace_back(st->open[cls], e);
  st->open[cls] = nullptr;
}

void tt_prof_free(tt_plan_s* p) {
  if (!p->prof) return;
  ProfState* st = static_cast<ProfState*>(p->prof);
  for (auto& v : st->done)
    for (auto& pr : v) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
  delete st;
  p->prof = nullptr;
}

extern "C" {

tt_status tt_plan_profile(tt_plan p, int32_t enable) {
  if (!p) return tt_fail(TT_ERR_ARG, "null plan");
  if (enable && !p->prof) p->prof = new ProfState();
  if (!enable) tt_prof_free(p);
  return TT_OK;
}

tt_status tt_plan_profile_read(tt_plan p, int32_t nclass, double* ms, int64_t* launches) {
  if (!p || !ms || !launches || nclass < 0 || nclass > TT_PROF_NCLASS) return tt_fail(TT_ERR_ARG, "bad argument");
  for (int c = 0; c < nclass; ++c) {
    ms[c] = 0.0;
    launches[c] = 0;
  }
  if (!p->prof) return TT_OK;
  TT_HIP_TRY(hipStreamSynchronize(p->stream));
  ProfState* st = static_cast<ProfState*>(p->prof);
  for (int c = 0; c < TT_PROF_NCLASS; ++c) {
    for (auto& pr : st->done[c]) {
      float t = 0.f;
      if (c < nclass && hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) {
        ms[c] += t;
        launches[c] += 1;
      }
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
    st->done[c].clear();
  }
  return TT_OK;
}

}  // extern "C"
