// Autotuner of the batch path (mapa_autotune): times candidate launch
// settings of the enumeration on a representative batch and keeps the
// fastest.  The settings are the prefix split (smallest prefix-item size
// considered and the smallest mean item size a batch may take), the block
// shape of the persistent enumeration kernel (threads per block, blocks per
// compute unit) and the widest last-two-positions table it is built with.
// Results never depend on these settings; the tuner checks that every
// candidate returns exactly the first candidate's results.
#include <algorithm>
#include <cstring>
#include <vector>

#include "ctx.h"

using namespace mapa;

namespace {

struct Knob {
  int32_t mapa_tuning::*field;
  std::vector<int32_t> values;
};

}  // namespace

extern "C" int32_t mapa_autotune(mapa_ctx *c, const mapa_query *q, int32_t nq, int32_t reps,
                                 mapa_tuning *best_out, mapa_tune_trial *trials, int32_t cap,
                                 int32_t *ntrials) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (c->serve) return fail(MAPA_ERR_STATE, "mapa_autotune: the serving loop owns the context");
  if (nq < 1 || !q) return fail(MAPA_ERR_INVALID_ARG, "mapa_autotune needs at least one query");
  if (reps < 1 || reps > 100) return fail(MAPA_ERR_INVALID_ARG, "reps outside 1..100");
  if (cap < 0 || (cap > 0 && !trials)) return fail(MAPA_ERR_INVALID_ARG, "bad trials array");
  if (ntrials) *ntrials = 0;
  std::vector<mapa_query> hq(q, q + nq);
  for (auto &x : hq) x.commit = 0;  // tuning runs never change server state
  if (int32_t r = validate_queries(c, hq.data(), nq)) return r;
  if (!c->has_device) return fail(MAPA_ERR_NO_DEVICE, "context has no device");
  MAPA_HIPCHK(hipSetDevice(c->device));
  int32_t rc = sync_ctx(c);
  if (rc) return rc;
  mapa_query *d_q = nullptr;
  mapa_result *d_res = nullptr;
  if (dev_alloc(&d_q, (size_t)nq) != hipSuccess || dev_alloc(&d_res, (size_t)nq) != hipSuccess) {
    dev_free(d_q);
    dev_free(d_res);
    return fail(MAPA_ERR_OOM, "mapa_autotune: device buffers");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const mapa_tuning start = c->tuning;
  std::vector<mapa_result> ref((size_t)nq), got((size_t)nq);
  int32_t n_trials = 0;
  int32_t err = MAPA_OK;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dev_free(d_q);
    dev_free(d_res);
  };
  if (hipMemcpy(d_q, hq.data(), nq * sizeof(mapa_query), hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(MAPA_ERR_DEVICE, "mapa_autotune: setup");
  }
  // mean batch time of one setting, its results checked against the first
  auto time_one = [&](const mapa_tuning &t, bool first, double *ms) -> int32_t {
    int32_t r = mapa_set_tuning(c, &t);
    if (r) return r;
    hipStream_t s = c->internal;
    r = mapa_query_batch(c, d_q, nq, d_res, MAPA_DEVICE_PTRS, s);  // warm-up
    if (r) return r;
    MAPA_HIPCHK(hipEventRecord(e0, s));
    for (int32_t i = 0; i < reps; ++i) {
      r = mapa_query_batch(c, d_q, nq, d_res, MAPA_DEVICE_PTRS, s);
      if (r) return r;
    }
    MAPA_HIPCHK(hipEventRecord(e1, s));
    MAPA_HIPCHK(hipEventSynchronize(e1));
    float f = 0;
    MAPA_HIPCHK(hipEventElapsedTime(&f, e0, e1));
    *ms = (double)f / reps;
    std::vector<mapa_result> &dst = first ? ref : got;
    MAPA_HIPCHK(hipMemcpy(dst.data(), d_res, nq * sizeof(mapa_result), hipMemcpyDeviceToHost));
    if (!first && std::memcmp(ref.data(), got.data(), nq * sizeof(mapa_result)) != 0)
      return fail(MAPA_ERR_DEVICE, "mapa_autotune: results changed with the tuning");
    if (trials && n_trials < cap) trials[n_trials] = {t, *ms};
    ++n_trials;
    return MAPA_OK;
  };
  std::vector<Knob> knobs = {
      {&mapa_tuning::min_leaves_per_item, {16, 64, 256, 1024, 4096}},
      {&mapa_tuning::mean_item_leaves, {32, 128, 512, 2048, 8192}},
      {&mapa_tuning::threads_per_block, {64, 128, 192, 256}},
      {&mapa_tuning::blocks_per_cu, {0, 1, 2, 4, 8}},
  };
  if (c->wpr == 1) knobs.push_back({&mapa_tuning::pair_width, {0, -1, 6, 12}});
  mapa_tuning best = start;
  double best_ms = 0;
  err = time_one(best, true, &best_ms);
  // coordinate descent, two passes over the knobs
  for (int pass = 0; pass < 2 && !err; ++pass) {
    bool moved = false;
    for (const Knob &k : knobs) {
      for (int32_t v : k.values) {
        if (best.*(k.field) == v) continue;
        mapa_tuning t = best;
        t.*(k.field) = v;
        double ms = 0;
        err = time_one(t, false, &ms);
        if (err) break;
        if (ms < best_ms * 0.99) {  // keep a change only if it is clearly faster
          best = t;
          best_ms = ms;
          moved = true;
        }
      }
      if (err) break;
    }
    if (!moved) break;
  }
  cleanup();
  if (err) {
    (void)mapa_set_tuning(c, &start);
    return err;
  }
  rc = mapa_set_tuning(c, &best);
  if (rc) return rc;
  if (best_out) *best_out = best;
  if (ntrials) *ntrials = n_trials;
  return MAPA_OK;
}
