// serve.hip -- the serving runtime of bitbox_serve.h: a device-memory arena
// (host bookkeeping over offsets), FIFO admission under the arena budget, and
// continuous batching: every launch takes the admitted jobs waiting at that
// moment (compress jobs as one batched compress, then the decompress jobs),
// runs on one of several HIP streams, and retires when its event completes.
// The compute is the C ABI of bitbox.h; nothing here touches job data.
#include <math.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "bbx_internal.h"
#include "bitbox_serve.h"

// ---------------------------------------------------------------- arena

struct bbx_arena {
  size_t size = 0, align = 256, used = 0;
  std::map<size_t, size_t> free_;  // offset -> length, disjoint, never adjacent
  std::map<size_t, size_t> live_;  // offset -> length
};

static size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

extern "C" bbx_status bbx_arena_create(size_t bytes, size_t align, bbx_arena** out) {
  if (!out || align == 0 || (align & (align - 1)))
    return bbx::set_error(BBX_EINVAL, "arena: out is NULL or align is not a power of two");
  bbx_arena* a = new (std::nothrow) bbx_arena;
  if (!a) return bbx::set_error(BBX_ENOMEM, "arena: host allocation failed");
  a->align = align;
  a->size = bytes / align * align;
  if (a->size) a->free_[0] = a->size;
  *out = a;
  return BBX_OK;
}

extern "C" void bbx_arena_destroy(bbx_arena* a) { delete a; }

extern "C" bbx_status bbx_arena_alloc(bbx_arena* a, size_t bytes, size_t* offset) {
  if (!a || !offset) return bbx::set_error(BBX_EINVAL, "arena: NULL argument");
  const size_t need = round_up(bytes ? bytes : 1, a->align);
  auto best = a->free_.end();
  for (auto it = a->free_.begin(); it != a->free_.end(); ++it)
    if (it->second >= need && (best == a->free_.end() || it->second < best->second)) best = it;
  if (best == a->free_.end()) return bbx::set_error(BBX_ENOMEM, "arena: no free range fits");
  const size_t off = best->first, len = best->second;
  a->free_.erase(best);
  if (len > need) a->free_[off + need] = len - need;
  a->live_[off] = need;
  a->used += need;
  *offset = off;
  return BBX_OK;
}

extern "C" bbx_status bbx_arena_free(bbx_arena* a, size_t offset) {
  if (!a) return bbx::set_error(BBX_EINVAL, "arena: NULL argument");
  auto it = a->live_.find(offset);
  if (it == a->live_.end()) return bbx::set_error(BBX_EINVAL, "arena: no block starts at this offset");
  size_t off = it->first, len = it->second;
  a->live_.erase(it);
  a->used -= len;
  auto nx = a->free_.lower_bound(off);
  if (nx != a->free_.end() && nx->first == off + len) {  // merge with the next free range
    len += nx->second;
    nx = a->free_.erase(nx);
  }
  if (nx != a->free_.begin()) {  // merge with the previous free range
    auto pv = std::prev(nx);
    if (pv->first + pv->second == off) {
      off = pv->first;
      len += pv->second;
      a->free_.erase(pv);
    }
  }
  a->free_[off] = len;
  return BBX_OK;
}

extern "C" void bbx_arena_stats(const bbx_arena* a, size_t* used, size_t* free_total,
                                size_t* largest_free, size_t* free_ranges) {
  size_t ft = 0, lf = 0;
  if (a)
    for (const auto& kv : a->free_) {
      ft += kv.second;
      if (kv.second > lf) lf = kv.second;
    }
  if (used) *used = a ? a->used : 0;
  if (free_total) *free_total = ft;
  if (largest_free) *largest_free = lf;
  if (free_ranges) *free_ranges = a ? a->free_.size() : 0;
}

// ---------------------------------------------------------------- server

namespace {

constexpr size_t kResultHead = 256;  // status u32 at 0, size u64 at 8, result from 256
constexpr uint32_t kMaxStreams = 8;

struct Job {
  uint64_t id = 0;
  uint32_t kind = 0;  // 0 compress, 1 decompress
  uint32_t state = BBX_JOB_QUEUED;
  // compress
  const void* pos = nullptr;
  uint64_t n = 0;
  uint32_t dims = 3;
  bbx_dtype dtype = BBX_F32;
  double eb = 0.0;
  bbx_params prm{};
  // decompress
  const void* stream = nullptr;
  size_t stream_size = 0;
  uint8_t header[128];
  bbx_layout layout = BBX_AOS;
  // memory
  size_t res_off = 0, res_bytes = 0;  // result region (head + result)
  size_t result_cap = 0;              // bytes after the head
  size_t ws_need = 0;                 // workspace of the job alone
  // timing
  double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
  uint32_t batch_jobs = 0;
  bool fetched = false;
  uint32_t status = 0;
  uint64_t bytes = 0;
};

struct Launch {
  bool live = false;
  std::vector<uint64_t> jobs;
  size_t ws_off = 0;
  bool has_ws = false;
  hipEvent_t done = nullptr;
};

}  // namespace

struct bbx_server {
  bbx_server_config cfg{};
  uint8_t* base = nullptr;
  bbx_arena* arena = nullptr;
  size_t reserved = 0;  // workspace bytes promised to admitted, unlaunched jobs
  uint64_t next_id = 1;
  uint64_t launches = 0;
  std::deque<uint64_t> queue;  // submitted, not admitted (FIFO)
  std::deque<uint64_t> ready;  // admitted, not launched (FIFO)
  std::deque<uint64_t> done;   // finished, not yet popped
  uint32_t admitted_live = 0;  // admitted and not released
  uint32_t running = 0;
  std::unordered_map<uint64_t, Job> jobs;
  hipStream_t streams[kMaxStreams] = {};
  Launch slots[kMaxStreams];
  hipStream_t query = nullptr;
  std::chrono::steady_clock::time_point t0;
  std::vector<bbx_set> sets;  // scratch for launch building
};

static double now_of(const bbx_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

extern "C" double bbx_server_now(const bbx_server* s) { return s ? now_of(s) : 0.0; }

extern "C" bbx_status bbx_server_create(const bbx_server_config* cfg, void* d_arena,
                                        size_t arena_bytes, bbx_server** out) {
  if (!cfg || !out || !d_arena) return bbx::set_error(BBX_EINVAL, "server: NULL argument");
  if ((uintptr_t)d_arena & 255) return bbx::set_error(BBX_EINVAL, "server: arena must be 256-byte aligned");
  if (cfg->hbm_budget == 0 || cfg->hbm_budget > arena_bytes)
    return bbx::set_error(BBX_EINVAL, "server: hbm_budget must be in (0, arena_bytes]");
  if (cfg->max_jobs == 0 || cfg->max_batch == 0 || cfg->nstreams == 0 || cfg->nstreams > kMaxStreams)
    return bbx::set_error(BBX_EINVAL, "server: max_jobs, max_batch >= 1 and nstreams in 1..8");
  if (cfg->tile_override != 0 && cfg->tile_override != 256 && cfg->tile_override != 512)
    return bbx::set_error(BBX_EINVAL, "server: tile_override must be 0, 256 or 512");
  bbx_server* s = new (std::nothrow) bbx_server;
  if (!s) return bbx::set_error(BBX_ENOMEM, "server: host allocation failed");
  s->cfg = *cfg;
  s->base = (uint8_t*)d_arena;
  s->t0 = std::chrono::steady_clock::now();
  bbx_status st = bbx_arena_create(cfg->hbm_budget, 256, &s->arena);
  hipError_t e = hipSuccess;
  for (uint32_t i = 0; st == BBX_OK && e == hipSuccess && i < cfg->nstreams; ++i) {
    e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->slots[i].done, hipEventDisableTiming);
  }
  if (st == BBX_OK && e == hipSuccess) e = hipStreamCreateWithFlags(&s->query, hipStreamNonBlocking);
  if (st != BBX_OK || e != hipSuccess) {
    bbx_server_destroy(s);
    return st != BBX_OK ? st : bbx::set_error(BBX_EHIP, hipGetErrorString(e));
  }
  *out = s;
  return BBX_OK;
}

extern "C" bbx_status bbx_server_destroy(bbx_server* s) {
  if (!s) return BBX_OK;
  for (uint32_t i = 0; i < kMaxStreams; ++i) {
    if (s->streams[i]) {
      (void)hipStreamSynchronize(s->streams[i]);
      (void)hipStreamDestroy(s->streams[i]);
    }
    if (s->slots[i].done) (void)hipEventDestroy(s->slots[i].done);
  }
  if (s->query) (void)hipStreamDestroy(s->query);
  bbx_arena_destroy(s->arena);
  delete s;
  return BBX_OK;
}

static bbx_status enqueue(bbx_server* s, Job& j, uint64_t* id) {
  size_t used, ft, lf, nr;
  bbx_arena_stats(s->arena, &used, &ft, &lf, &nr);
  const size_t need = round_up(j.res_bytes, 256) + round_up(j.ws_need, 256);
  if (need > s->arena->size) return bbx::set_error(BBX_ENOMEM, "server: job exceeds the whole budget");
  j.id = s->next_id++;
  j.t_submit = now_of(s);
  s->queue.push_back(j.id);
  s->jobs.emplace(j.id, j);
  *id = j.id;
  return BBX_OK;
}

extern "C" bbx_status bbx_server_submit_compress(bbx_server* s, const void* d_pos, uint64_t n,
                                                 uint32_t dims, bbx_dtype dtype, double eb,
                                                 const bbx_params* params, uint64_t* job) {
  if (!s || !job || !params) return bbx::set_error(BBX_EINVAL, "server: NULL argument");
  bbx_params p = *params;
  p.tile_override = s->cfg.tile_override;  // one tile per launch
  p.scatter_stage = 0;                     // the library's choice: jobs of a launch share it
  p.level_blocks = 0;                      // the library's choice (the set's share of the launch)
  const size_t ws = bbx_compress_workspace_size(n, dims, dtype, &p);
  if (ws == 0) return bbx_compress(d_pos, n, dims, dtype, eb, &p, nullptr, 0, nullptr, nullptr,
                                   nullptr, nullptr, nullptr, 0, nullptr);  // its argument error
  if (!isfinite(eb) || !(eb > 0.0)) return bbx::set_error(BBX_EINVAL, "eb must be finite and > 0");
  if (n > 0 && !d_pos) return bbx::set_error(BBX_EINVAL, "positions pointer is NULL");
  Job j;
  j.kind = 0;
  j.pos = d_pos;
  j.n = n;
  j.dims = dims;
  j.dtype = dtype;
  j.eb = eb;
  j.prm = p;
  j.result_cap = round_up(bbx_compress_bound_params(n, dims, dtype, &p), 8);
  j.res_bytes = kResultHead + j.result_cap;
  j.ws_need = ws;
  return enqueue(s, j, job);
}

extern "C" bbx_status bbx_server_submit_decompress(bbx_server* s, const void* d_stream,
                                                   size_t stream_size, const void* h_header,
                                                   bbx_layout layout, uint64_t* job) {
  if (!s || !job || !h_header || !d_stream) return bbx::set_error(BBX_EINVAL, "server: NULL argument");
  if (layout != BBX_AOS && layout != BBX_SOA) return bbx::set_error(BBX_EINVAL, "layout must be AOS or SOA");
  uint64_t n = 0, nl = 0, sb = 0;
  uint32_t dims = 0, r = 0;
  bbx_dtype dt;
  double eba;
  bbx_status st = bbx_stream_info(h_header, 128, &n, &dims, &dt, &eba, &r, &nl, &sb);
  if (st != BBX_OK) return st;
  if (sb > stream_size) return bbx::set_error(BBX_ECORRUPT, "stream shorter than its header says");
  const size_t ws = bbx_decompress_workspace_size(h_header, 128);
  if (ws == 0) return bbx::set_error(BBX_ECORRUPT, "stream header rejected");
  Job j;
  j.kind = 1;
  j.stream = d_stream;
  j.stream_size = stream_size;
  memcpy(j.header, h_header, 128);
  j.layout = layout;
  j.n = n;
  j.dims = dims;
  j.dtype = dt;
  j.result_cap = round_up((size_t)n * dims * (dt == BBX_F32 ? 4 : 8), 8);
  j.res_bytes = kResultHead + j.result_cap;
  j.ws_need = ws;
  return enqueue(s, j, job);
}

// FIFO admission: the head job enters when its result region can be placed
// and the free space left still covers every promised workspace plus its own.
static void admit(bbx_server* s) {
  while (!s->queue.empty() && s->admitted_live < s->cfg.max_jobs) {
    Job& j = s->jobs[s->queue.front()];
    size_t used, ft, lf, nr;
    bbx_arena_stats(s->arena, &used, &ft, &lf, &nr);
    const size_t wsr = round_up(j.ws_need, 256);
    if (ft < round_up(j.res_bytes, 256) + s->reserved + wsr) break;
    size_t off;
    if (bbx_arena_alloc(s->arena, j.res_bytes, &off) != BBX_OK) break;
    bbx_arena_stats(s->arena, &used, &ft, &lf, &nr);
    if (lf < wsr) {  // its workspace could not be placed now: wait for memory
      (void)bbx_arena_free(s->arena, off);
      break;
    }
    j.res_off = off;
    j.state = BBX_JOB_ADMITTED;
    j.t_admit = now_of(s);
    s->reserved += wsr;
    s->admitted_live++;
    s->ready.push_back(j.id);
    s->queue.pop_front();
  }
}

static void retire(bbx_server* s, uint32_t* n_done) {
  for (uint32_t i = 0; i < s->cfg.nstreams; ++i) {
    Launch& L = s->slots[i];
    if (!L.live) continue;
    if (hipEventQuery(L.done) != hipSuccess) continue;  // hipErrorNotReady: still running
    const double t = now_of(s);
    for (uint64_t id : L.jobs) {
      Job& j = s->jobs[id];
      j.state = BBX_JOB_DONE;
      j.t_done = t;
      s->done.push_back(id);
      s->running--;
      if (n_done) (*n_done)++;
    }
    if (L.has_ws) (void)bbx_arena_free(s->arena, L.ws_off);
    L.jobs.clear();
    L.has_ws = false;
    L.live = false;
  }
}

// Workspace layout of a launch: the batched compress first, then one region
// per decompress job.
static size_t launch_ws(bbx_server* s, const std::vector<uint64_t>& ids, size_t* ws_c,
                        std::vector<size_t>* ws_d) {
  s->sets.clear();
  ws_d->clear();
  size_t total = 0;
  for (uint64_t id : ids) {
    Job& j = s->jobs[id];
    if (j.kind == 0) {
      bbx_set st;
      memset(&st, 0, sizeof(st));
      uint8_t* res = s->base + j.res_off;
      st.d_pos = j.pos;
      st.n = j.n;
      st.dims = j.dims;
      st.dtype = (uint32_t)j.dtype;
      st.eb = j.eb;
      st.params = j.prm;
      st.d_out = res + kResultHead;
      st.out_cap = j.result_cap;
      st.d_status = (uint32_t*)res;
      st.d_size = (uint64_t*)(res + 8);
      st.d_perm = nullptr;
      s->sets.push_back(st);
    } else {
      ws_d->push_back(round_up(j.ws_need, 256));
      total += ws_d->back();
    }
  }
  *ws_c = s->sets.empty() ? 0 : round_up(bbx_batch_workspace_size(s->sets.data(), (uint32_t)s->sets.size()), 256);
  return total + *ws_c;
}

static bbx_status start_launch(bbx_server* s, uint32_t slot) {
  std::vector<uint64_t> ids;
  for (size_t k = 0; k < s->ready.size() && ids.size() < s->cfg.max_batch; ++k)
    ids.push_back(s->ready[k]);
  size_t ws_c = 0, off = 0;
  std::vector<size_t> ws_d;
  for (;;) {  // the launch's workspace must fit; drop the newest jobs until it does
    const size_t total = launch_ws(s, ids, &ws_c, &ws_d);
    if (bbx_arena_alloc(s->arena, total, &off) == BBX_OK) break;
    if (ids.size() == 1) return BBX_ENOMEM;  // wait for a retirement
    ids.resize(ids.size() / 2);
  }
  Launch& L = s->slots[slot];
  hipStream_t st = s->streams[slot];
  uint8_t* ws = s->base + off;
  bbx_status rc = BBX_OK;
  if (!s->sets.empty()) {
    rc = bbx_compress_batch(s->sets.data(), (uint32_t)s->sets.size(), ws, ws_c, st);
  }
  size_t at = ws_c, di = 0;
  for (uint64_t id : ids) {
    Job& j = s->jobs[id];
    if (j.kind != 1 || rc != BBX_OK) continue;
    uint8_t* res = s->base + j.res_off;
    rc = bbx_decompress(j.stream, j.stream_size, j.header, res + kResultHead, j.result_cap,
                        j.layout, (uint32_t*)res, ws + at, ws_d[di], st);
    at += ws_d[di++];
  }
  if (rc == BBX_OK) {
    hipError_t e = hipEventRecord(L.done, st);
    if (e != hipSuccess) rc = bbx::set_error(BBX_EHIP, hipGetErrorString(e));
  }
  if (rc != BBX_OK) {  // argument errors were screened at submit: not expected
    (void)hipStreamSynchronize(st);
    (void)bbx_arena_free(s->arena, off);
    return rc;
  }
  const double t = now_of(s);
  for (uint64_t id : ids) {
    Job& j = s->jobs[id];
    j.state = BBX_JOB_RUNNING;
    j.t_launch = t;
    j.batch_jobs = (uint32_t)ids.size();
    s->reserved -= round_up(j.ws_need, 256);
    s->running++;
  }
  s->ready.erase(s->ready.begin(), s->ready.begin() + ids.size());
  L.jobs = ids;
  L.ws_off = off;
  L.has_ws = true;
  L.live = true;
  s->launches++;
  return BBX_OK;
}

extern "C" bbx_status bbx_server_progress(bbx_server* s, uint32_t* n_done) {
  if (!s) return bbx::set_error(BBX_EINVAL, "server: NULL argument");
  if (n_done) *n_done = 0;
  retire(s, n_done);
  admit(s);
  for (uint32_t i = 0; i < s->cfg.nstreams && !s->ready.empty(); ++i) {
    if (s->slots[i].live) continue;
    bbx_status rc = start_launch(s, i);
    if (rc == BBX_ENOMEM) break;
    if (rc != BBX_OK) return rc;
  }
  return BBX_OK;
}

extern "C" uint64_t bbx_server_pop_done(bbx_server* s) {
  if (!s || s->done.empty()) return 0;
  const uint64_t id = s->done.front();
  s->done.pop_front();
  return id;
}

extern "C" bbx_status bbx_server_job_info(bbx_server* s, uint64_t job, bbx_job_info* info) {
  if (!s || !info) return bbx::set_error(BBX_EINVAL, "server: NULL argument");
  auto it = s->jobs.find(job);
  if (it == s->jobs.end()) return bbx::set_error(BBX_EINVAL, "server: unknown or released job");
  Job& j = it->second;
  if (j.state == BBX_JOB_DONE && !j.fetched) {
    uint64_t head[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(head, s->base + j.res_off, 16, hipMemcpyDeviceToHost, s->query);
    if (e == hipSuccess) e = hipStreamSynchronize(s->query);
    if (e != hipSuccess) return bbx::set_error(BBX_EHIP, hipGetErrorString(e));
    j.status = (uint32_t)head[0];
    if (j.status != BBX_OK)
      j.bytes = 0;
    else
      j.bytes = j.kind == 0 ? head[1] : (uint64_t)j.n * j.dims * (j.dtype == BBX_F32 ? 4 : 8);
    j.fetched = true;
  }
  info->state = j.state;
  info->status = j.fetched ? j.status : 0;
  info->bytes = j.fetched ? j.bytes : 0;
  info->d_result = j.state >= BBX_JOB_ADMITTED ? (void*)(s->base + j.res_off + kResultHead) : nullptr;
  info->t_submit = j.t_submit;
  info->t_admit = j.t_admit;
  info->t_launch = j.t_launch;
  info->t_done = j.t_done;
  info->batch_jobs = j.batch_jobs;
  info->kind = j.kind;
  return BBX_OK;
}

extern "C" bbx_status bbx_server_release(bbx_server* s, uint64_t job) {
  if (!s) return bbx::set_error(BBX_EINVAL, "server: NULL argument");
  auto it = s->jobs.find(job);
  if (it == s->jobs.end()) return bbx::set_error(BBX_EINVAL, "server: unknown or released job");
  if (it->second.state != BBX_JOB_DONE) return bbx::set_error(BBX_EINVAL, "server: job not finished");
  (void)bbx_arena_free(s->arena, it->second.res_off);
  s->admitted_live--;
  s->jobs.erase(it);
  return BBX_OK;
}

extern "C" void bbx_server_counts(const bbx_server* s, uint32_t* queued, uint32_t* admitted,
                                  uint32_t* running, uint32_t* inflight, uint64_t* launches,
                                  size_t* arena_used) {
  uint32_t fl = 0;
  if (s)
    for (uint32_t i = 0; i < s->cfg.nstreams; ++i) fl += s->slots[i].live ? 1u : 0u;
  if (queued) *queued = s ? (uint32_t)s->queue.size() : 0;
  if (admitted) *admitted = s ? (uint32_t)s->ready.size() : 0;
  if (running) *running = s ? s->running : 0;
  if (inflight) *inflight = fl;
  if (launches) *launches = s ? s->launches : 0;
  if (arena_used) *arena_used = s && s->arena ? s->arena->used : 0;
}
