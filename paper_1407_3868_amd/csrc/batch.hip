// Batches of matvecs over several contexts (configurations), captured once
// into one HIP graph with a parallel branch per item and replayed with a
// single graph launch.
#include <vector>

#include "kernels.h"

struct mpsl_batch {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<mpsl_ctx *> ctxs;  // pinned while the batch exists
  int device = 0;
  std::string err;
};

namespace {

void batch_free(mpsl_batch *b) {
  if (!b) return;
  for (auto c : b->ctxs) --c->pinned;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto s : b->streams) (void)hipStreamDestroy(s);
  for (auto e : b->events) (void)hipEventDestroy(e);
  delete b;
}

}  // namespace

extern "C" {

int mpsl_batch_create(mpsl_batch **out, int n_items, mpsl_ctx *const *ctxs, const int *precs, const int *nrhs,
                      const void *const *x, void *const *y) {
  if (!out || n_items <= 0 || !ctxs || !precs || !x || !y) return MPSL_EINVAL;
  *out = nullptr;
  const int dev = ctxs[0]->device;
  for (int i = 0; i < n_items; ++i) {
    if (!ctxs[i] || !x[i] || !y[i] || (precs[i] != MPSL_FP64 && precs[i] != MPSL_FP32) ||
        (nrhs && nrhs[i] < 1) || ctxs[i]->device != dev)
      return MPSL_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i])
        return mpsl::set_err(ctxs[i], MPSL_EINVAL, "a context appears twice in one batch (its work buffers are shared)");
  }
  if (hipSetDevice(dev) != hipSuccess) return MPSL_EHIP;
  // warm-up: builds tables and sizes every work buffer, so that nothing is
  // allocated while the graph is captured
  for (int i = 0; i < n_items; ++i) {
    const int rc = mpsl::matvec(ctxs[i], precs[i], x[i], y[i], nrhs ? nrhs[i] : 1);
    if (rc) return rc;
    if (hipStreamSynchronize(ctxs[i]->stream) != hipSuccess) return MPSL_EHIP;
  }
  mpsl_batch *b = new mpsl_batch();
  b->device = dev;
  hipStream_t root;
  if (hipStreamCreateWithFlags(&root, hipStreamNonBlocking) != hipSuccess) {
    batch_free(b);
    return MPSL_EHIP;
  }
  b->streams.push_back(root);
  hipEvent_t fork;
  if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) {
    batch_free(b);
    return MPSL_EHIP;
  }
  b->events.push_back(fork);
  std::vector<hipStream_t> saved(n_items);
  std::vector<bool> saved_prof(n_items);
  int rc = MPSL_OK;
  if (hipStreamBeginCapture(root, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    batch_free(b);
    return MPSL_EHIP;
  }
  bool ok = hipEventRecord(fork, root) == hipSuccess;
  for (int i = 0; i < n_items && ok && !rc; ++i) {
    hipStream_t s;
    hipEvent_t join;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
      ok = false;
      break;
    }
    b->streams.push_back(s);
    b->events.push_back(join);
    ok = hipStreamWaitEvent(s, fork, 0) == hipSuccess;
    saved[i] = ctxs[i]->stream;
    saved_prof[i] = ctxs[i]->prof;
    ctxs[i]->stream = s;
    ctxs[i]->prof = false;
    if (ok) rc = mpsl::matvec(ctxs[i], precs[i], x[i], y[i], nrhs ? nrhs[i] : 1);
    ctxs[i]->stream = saved[i];
    ctxs[i]->prof = saved_prof[i];
    ok = ok && hipEventRecord(join, s) == hipSuccess && hipStreamWaitEvent(root, join, 0) == hipSuccess;
  }
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(root, &g);
  if (!ok || rc || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    batch_free(b);
    (void)hipGetLastError();
    return rc ? rc : MPSL_EHIP;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    batch_free(b);
    return MPSL_EHIP;
  }
  // the graph holds the addresses of every item's tables and work buffers
  for (int i = 0; i < n_items; ++i) {
    b->ctxs.push_back(ctxs[i]);
    ++ctxs[i]->pinned;
  }
  *out = b;
  return MPSL_OK;
}

int mpsl_batch_launch(mpsl_batch *b, void *stream) {
  if (!b) return MPSL_EINVAL;
  if (hipSetDevice(b->device) != hipSuccess) return MPSL_EHIP;
  if (hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)) != hipSuccess) return MPSL_EHIP;
  return MPSL_OK;
}

void mpsl_batch_destroy(mpsl_batch *b) { batch_free(b); }

}  // extern "C"
