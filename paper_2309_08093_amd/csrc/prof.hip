// Opt-in per-kernel-class timing with HIP events on the plan's stream.
#include <utility>
#include <vector>

#include "tt_internal.h"

namespace {
struct ProfState {
  uint32_t mask = 0;   // classes timed (bit c for class c)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> done[TT_PROF_NCLASS];
  hipEvent_t open[TT_PROF_NCLASS] = {};
  std::vector<hipEvent_t> pool;   // events of earlier reads, recorded again

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
  }
};

bool timed(const tt_plan_s* p, int cls) {
  return p->prof && ((static_cast<ProfState*>(p->prof)->mask >> cls) & 1u);
}
}  // namespace

void tt_prof_begin(const tt_plan_s* p, int cls) {
  if (!timed(p, cls)) return;
  ProfState* st = static_cast<ProfState*>(p->prof);
  hipEvent_t e = st->take();
  if (!e) return;
  hipEventRecord(e, p->stream);
  st->open[cls] = e;
}

void tt_prof_end(const tt_plan_s* p, int cls) {
  if (!timed(p, cls)) return;
  ProfState* st = static_cast<ProfState*>(p->prof);
  if (!st->open[cls]) return;
  hipEvent_t e = st->take();
  if (!e) return;
  hipEventRecord(e, p->stream);
  st->done[cls].emplace_back(st->open[cls], e);
  st->open[cls] = nullptr;
}

void tt_prof_free(tt_plan_s* p) {
  if (!p->prof) return;
  ProfState* st = static_cast<ProfState*>(p->prof);
  (void)hipStreamSynchronize(p->stream);
  for (auto& v : st->done)
    for (auto& pr : v) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : st->open)
    if (e) hipEventDestroy(e);
  for (hipEvent_t e : st->pool) hipEventDestroy(e);
  delete st;
  p->prof = nullptr;
}

extern "C" {

tt_status tt_plan_profile(tt_plan p, int32_t enable) {
  if (!p) return tt_fail(TT_ERR_ARG, "null plan");
  if (!enable) {
    tt_prof_free(p);
    return TT_OK;
  }
  if (!p->prof) p->prof = new ProfState();
  static_cast<ProfState*>(p->prof)->mask = (uint32_t)enable;
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
      st->pool.push_back(pr.first);
      st->pool.push_back(pr.second);
    }
    st->done[c].clear();
  }
  return TT_OK;
}

}  // extern "C"
