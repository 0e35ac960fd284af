// Serving several concurrent sensor streams on one GPU.
//
// The method is meant to keep up with a sensor in real time (the frame-rate
// budget of Section 3.6); a server applies that to several sensors at once.
// Each admitted stream owns a context (its TSDF, points and labels stay in
// device memory between frames), a HIP stream, a recorded frame graph
// (integration followed by scoring of the stream's tools) and a small queue
// of pinned host slots that hold frames as they arrive.  One step takes the
// oldest queued frame of every stream and launches each stream's recorded
// frame on its own HIP stream, where the GPU overlaps them.  In batched mode
// (af_server_batch) the graphs stop after the candidate masks, and when
// enough streams took a frame one scoring launch labels the points of all
// of them, each against its own map and tools, after which every stream
// reads its counts back; fewer streams are scored each on its own stream.
// Otherwise (the default) each stream's graph also holds its own scoring
// launch.
//
// A stream whose context is in the incremental mode (Section 3.5) records
// no graph: its frames run af_incremental_frame on its own HIP stream, and a
// stream with a sliding window records its scoring inside its own graph;
// neither takes part in the batched scoring launch.
//
// Admission reserves the stream's declared device budget (af_config.
// hbm_budget) against the server's budget.  A context never allocates beyond
// its own budget, so the streams together never exceed the server's.
//
// Host code only: everything on the device is done by the context calls.

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <vector>

#include "af.h"
#include "af_internal.h"

namespace {

constexpr int kQueueSlots = 4;   // frames a stream may have waiting
constexpr int kMaxServed = 64;   // stream slots of one server

struct Slot {
  float *host;
  int64_t n;
  float origin[3];
  int64_t frame_id;
};

struct Served {
  bool used = false;
  af_ctx *ctx = nullptr;
  hipStream_t hs = nullptr;
  hipEvent_t done = nullptr;   // the stream's integration of this step (batched mode)
  std::vector<int32_t> tools;  // tools its frames are scored for
  bool batched = false;        // graph recorded without scoring
  bool incremental = false;    // frames run af_incremental_frame (no graph)
  int64_t reserved = 0;
  int64_t max_returns = 0;   // 0 until the frame graph is recorded
  int64_t last_id = -1;      // last frame id queued
  std::vector<float *> slots;
  std::vector<float *> free_slots;
  std::deque<Slot> queue;
};

}  // namespace

struct af_server {
  int64_t budget = 0;
  int64_t reserved = 0;
  int32_t rr = 0;   // stream visited first by the next step (round robin)
  std::vector<Served> streams;
  int32_t batch_min = 0;         // streams in a step that get one scoring launch (0: never)
  hipStream_t bs = nullptr;      // the batched scoring launch's stream
  hipEvent_t scored = nullptr;   // recorded after it
  af::ScoreJob *jobs_host = nullptr;   // pinned, kMaxJobs
  af::ScoreJob *jobs_dev = nullptr;
  unsigned *work = nullptr;
  char err[256] = "no error";
};

namespace {

int sfail(af_server *s, int rc, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(s->err, sizeof(s->err), fmt, ap);
  va_end(ap);
  return rc;
}

// The batched launch's stream, event, job tables and work counter (made on
// the first prepare in batched mode).
int batch_resources(af_server *s) {
  if (s->bs) return AF_OK;
  if (hipStreamCreateWithFlags(&s->bs, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->scored, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void **)&s->jobs_host, sizeof(af::ScoreJob) * af::kMaxJobs) != hipSuccess ||
      hipMalloc((void **)&s->jobs_dev, sizeof(af::ScoreJob) * af::kMaxJobs) != hipSuccess ||
      hipMalloc((void **)&s->work, 64) != hipSuccess)
    return sfail(s, AF_EDEVICE, "batched scoring resources");
  return AF_OK;
}

Served *get(af_server *s, int32_t id) {
  if (!s || id < 0 || id >= (int32_t)s->streams.size() || !s->streams[id].used) return nullptr;
  return &s->streams[id];
}

void free_slots(Served &t) {
  for (float *p : t.slots) hipHostFree(p);
  t.slots.clear();
  t.free_slots.clear();
  t.queue.clear();
}

}  // namespace

extern "C" {

int af_server_create(int64_t hbm_budget, int32_t max_streams, af_server **out) {
  if (!out) return AF_EINVAL;
  *out = nullptr;
  if (hbm_budget <= 0 || max_streams < 1 || max_streams > kMaxServed) return AF_EINVAL;
  af_server *s = new af_server();
  s->budget = hbm_budget;
  s->streams.resize(max_streams);
  *out = s;
  return AF_OK;
}

int af_server_batch(af_server *s, int32_t min_streams) {
  if (!s) return AF_EINVAL;
  if (min_streams < 0) return sfail(s, AF_EINVAL, "min_streams %d < 0", min_streams);
  for (const Served &t : s->streams)
    if (t.used && t.max_returns)
      return sfail(s, AF_EINVAL, "choose the mode before any stream is prepared");
  s->batch_min = min_streams == 1 ? 2 : min_streams;
  return AF_OK;
}

int af_server_release(af_server *s, int32_t id) {
  Served *t = get(s, id);
  if (!t) return s ? sfail(s, AF_EINVAL, "stream %d is not admitted", id) : AF_EINVAL;
  hipStreamSynchronize(t->hs);
  if (s->bs) hipStreamSynchronize(s->bs);
  af_destroy(t->ctx);
  hipStreamDestroy(t->hs);
  if (t->done) hipEventDestroy(t->done);
  free_slots(*t);
  s->reserved -= t->reserved;
  *t = Served();
  return AF_OK;
}

int af_server_destroy(af_server *s) {
  if (!s) return AF_EINVAL;
  for (int32_t i = 0; i < (int32_t)s->streams.size(); ++i)
    if (s->streams[i].used) af_server_release(s, i);
  if (s->bs) hipStreamSynchronize(s->bs);
  if (s->jobs_dev) hipFree(s->jobs_dev);
  if (s->work) hipFree(s->work);
  if (s->jobs_host) hipHostFree(s->jobs_host);
  if (s->scored) hipEventDestroy(s->scored);
  if (s->bs) hipStreamDestroy(s->bs);
  delete s;
  return AF_OK;
}

const char *af_server_last_error(af_server *s) { return s ? s->err : "null server"; }

int64_t af_server_reserved(af_server *s) { return s ? s->reserved : -1; }

int af_server_admit(af_server *s, const af_config *cfg, int32_t *id) {
  if (!s) return AF_EINVAL;
  if (!cfg || !id) return sfail(s, AF_EINVAL, "null configuration or id");
  *id = -1;
  if (cfg->hbm_budget <= 0)
    return sfail(s, AF_EINVAL, "a served stream must declare its device budget");
  if (cfg->hbm_budget > s->budget - s->reserved)
    return sfail(s, AF_ENOMEM, "stream needs %lld bytes, %lld of %lld left",
                 (long long)cfg->hbm_budget, (long long)(s->budget - s->reserved),
                 (long long)s->budget);
  int32_t slot = -1;
  for (int32_t i = 0; i < (int32_t)s->streams.size() && slot < 0; ++i)
    if (!s->streams[i].used) slot = i;
  if (slot < 0) return sfail(s, AF_EBUSY, "all %d stream slots in use", (int)s->streams.size());
  Served t;
  int rc = af_create(cfg, &t.ctx);
  if (rc != AF_OK) return sfail(s, rc, "context creation failed (%d)", rc);
  if (hipStreamCreateWithFlags(&t.hs, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&t.done, hipEventDisableTiming) != hipSuccess) {
    if (t.hs) hipStreamDestroy(t.hs);
    af_destroy(t.ctx);
    return sfail(s, AF_EDEVICE, "stream creation failed");
  }
  t.used = true;
  t.reserved = cfg->hbm_budget;
  s->reserved += t.reserved;
  s->streams[slot] = std::move(t);
  *id = slot;
  return AF_OK;
}

af_ctx *af_server_context(af_server *s, int32_t id) {
  Served *t = get(s, id);
  return t ? t->ctx : nullptr;
}

void *af_server_hip_stream(af_server *s, int32_t id) {
  Served *t = get(s, id);
  return t ? (void *)t->hs : nullptr;
}

int af_server_prepare(af_server *s, int32_t id, const float lo[3], const float hi[3],
                      int64_t max_returns, const int32_t *tool_ids, int32_t n_tools) {
  Served *t = get(s, id);
  if (!t) return s ? sfail(s, AF_EINVAL, "stream %d is not admitted", id) : AF_EINVAL;
  if (max_returns < 1 || max_returns > (int64_t)1 << 26)
    return sfail(s, AF_EINVAL, "max_returns %lld out of range", (long long)max_returns);
  hipStreamSynchronize(t->hs);
  free_slots(*t);
  t->max_returns = 0;
  const bool incremental = af::ctx_incremental(t->ctx);
  const bool batched = s->batch_min > 0 && !af::ctx_windowed(t->ctx) && !incremental;
  if (batched) {
    const int rc = batch_resources(s);
    if (rc != AF_OK) return rc;
  }
  int rc = incremental ? af::ctx_frame_slot(t->ctx, max_returns)
           : batched   ? af::ctx_graph_prepare_unscored(t->ctx, lo, hi, max_returns, tool_ids,
                                                        n_tools, t->hs)
                       : af_graph_prepare(t->ctx, lo, hi, max_returns, tool_ids, n_tools, t->hs);
  if (rc != AF_OK) return sfail(s, rc, "stream %d: %s", id, af_last_error(t->ctx));
  if (incremental) t->tools.clear();
  else t->tools.assign(tool_ids, tool_ids + n_tools);
  t->batched = batched;
  t->incremental = incremental;
  for (int i = 0; i < kQueueSlots; ++i) {
    float *p = nullptr;
    if (hipHostMalloc((void **)&p, sizeof(float) * 3 * max_returns) != hipSuccess) {
      free_slots(*t);
      return sfail(s, AF_ENOMEM, "pinned frame slots");
    }
    t->slots.push_back(p);
    t->free_slots.push_back(p);
  }
  t->max_returns = max_returns;
  return AF_OK;
}

int af_server_submit(af_server *s, int32_t id, const float *xyz, int64_t n,
                     const float origin[3], int64_t frame_id) {
  Served *t = get(s, id);
  if (!t) return s ? sfail(s, AF_EINVAL, "stream %d is not admitted", id) : AF_EINVAL;
  if (!t->max_returns) return sfail(s, AF_EINVAL, "stream %d has no recorded frame", id);
  if (n < 0 || n > t->max_returns || (n > 0 && !xyz) || !origin)
    return sfail(s, AF_EINVAL, "stream %d: bad frame (n = %lld)", id, (long long)n);
  if (frame_id <= t->last_id)
    return sfail(s, AF_EINVAL, "stream %d: frame id %lld does not increase", id,
                 (long long)frame_id);
  if (t->free_slots.empty()) return sfail(s, AF_EBUSY, "stream %d: %d frames waiting", id,
                                          kQueueSlots);
  Slot f;
  f.host = t->free_slots.back();
  t->free_slots.pop_back();
  if (n > 0) memcpy(f.host, xyz, sizeof(float) * 3 * n);
  f.n = n;
  memcpy(f.origin, origin, sizeof(f.origin));
  f.frame_id = frame_id;
  t->queue.push_back(f);
  t->last_id = frame_id;
  return AF_OK;
}

int32_t af_server_pending(af_server *s, int32_t id) {
  Served *t = get(s, id);
  return t ? (int32_t)t->queue.size() : -1;
}

int af_server_step(af_server *s, int32_t *stream_ids, int64_t *frame_ids, int32_t *status,
                   int32_t cap, int32_t *n_done) {
  if (!s) return AF_EINVAL;
  const int32_t ns = (int32_t)s->streams.size();
  if (!stream_ids || !frame_ids || !status || !n_done || cap < ns)
    return sfail(s, AF_EINVAL, "result arrays must hold %d entries", ns);
  *n_done = 0;
  struct Launched {
    int32_t id;
    int rc;
  };
  std::vector<Launched> run;
  for (int32_t k = 0; k < ns; ++k) {
    const int32_t id = (s->rr + k) % ns;
    Served &t = s->streams[id];
    if (!t.used || t.queue.empty()) continue;
    const Slot &f = t.queue.front();
    float *dev = af_graph_slot(t.ctx);
    int rc = AF_OK;
    if (f.n > 0 && hipMemcpyAsync(dev, f.host, sizeof(float) * 3 * f.n, hipMemcpyHostToDevice,
                                  t.hs) != hipSuccess)
      rc = AF_EDEVICE;
    if (rc == AF_OK)
      rc = t.incremental ? af_incremental_frame(t.ctx, dev, f.n, f.origin, f.frame_id, t.hs)
                         : af_graph_frame(t.ctx, dev, f.n, f.origin, f.frame_id, t.hs);
    run.push_back({id, rc});
  }
  s->rr = (s->rr + 1) % ns;
  // batched mode: one scoring launch over the streams that integrated a
  // frame when there are at least batch_min of them; otherwise (and past the
  // launch's job capacity) a stream is scored on its own stream, with no
  // cross-stream wait
  std::vector<int32_t> batch;
  for (Launched &l : run)
    if (l.rc == AF_OK && s->streams[l.id].batched) batch.push_back(l.id);
  int32_t n_jobs = 0;
  std::vector<char> in_launch(ns, 0);
  if (s->batch_min > 0 && (int32_t)batch.size() >= s->batch_min)
    for (int32_t id : batch) {
      Served &t = s->streams[id];
      if (n_jobs + (int32_t)t.tools.size() > af::kMaxJobs) continue;
      af::ctx_score_jobs(t.ctx, t.tools.data(), (int32_t)t.tools.size(), s->jobs_host + n_jobs);
      n_jobs += (int32_t)t.tools.size();
      in_launch[id] = 1;
      hipEventRecord(t.done, t.hs);
      hipStreamWaitEvent(s->bs, t.done, 0);
    }
  for (Launched &l : run)
    if (l.rc == AF_OK && s->streams[l.id].batched && !in_launch[l.id]) {
      Served &t = s->streams[l.id];
      l.rc = af::ctx_score_stream(t.ctx, t.tools.data(), (int32_t)t.tools.size(), t.hs);
    }
  int batch_rc = AF_OK;
  if (n_jobs > 0) {
    int32_t words = 0;
    for (int32_t j = 0; j < n_jobs; ++j) {
      s->jobs_host[j].base = words;
      words += s->jobs_host[j].t.K + 1;
    }
    if (hipMemcpyAsync(s->jobs_dev, s->jobs_host, sizeof(af::ScoreJob) * n_jobs,
                       hipMemcpyHostToDevice, s->bs) != hipSuccess ||
        af::launch_score_jobs(s->jobs_dev, s->jobs_host, n_jobs, s->work, s->bs) != 0 ||
        hipGetLastError() != hipSuccess)
      batch_rc = AF_EDEVICE;
    hipEventRecord(s->scored, s->bs);
    for (const Launched &l : run)
      if (in_launch[l.id]) hipStreamWaitEvent(s->streams[l.id].hs, s->scored, 0);
  }
  int worst = AF_OK;
  for (Launched &l : run) {
    Served &t = s->streams[l.id];
    int rc = l.rc;
    if (rc == AF_OK && in_launch[l.id] && batch_rc != AF_OK) {
      hipStreamSynchronize(t.hs);
      rc = batch_rc;
    }
    if (rc == AF_OK) rc = af_graph_sync(t.ctx);
    else hipStreamSynchronize(t.hs);   // the copy may still read the slot
    const Slot f = t.queue.front();
    t.queue.pop_front();
    t.free_slots.push_back(f.host);
    stream_ids[*n_done] = l.id;
    frame_ids[*n_done] = f.frame_id;
    status[*n_done] = rc;
    ++*n_done;
    if (rc != AF_OK && worst == AF_OK) {
      worst = rc;
      sfail(s, rc, "stream %d frame %lld: %s", l.id, (long long)f.frame_id,
            af_last_error(t.ctx));
    }
  }
  return AF_OK;
}

}  // extern "C"
