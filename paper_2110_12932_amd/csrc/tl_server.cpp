// Serving loop of the two-level thermal library: continuous batching of many
// independent simulations on one GPU.
//
// Requests (a mesh, material, scan path and options each) are queued by
// tl_server_submit.  Every tl_server_tick first admits queued requests in
// arrival order while a slot is free and the request's device footprint fits
// both the HBM budget and the caller's pool (a first-fit allocator with
// coalescing carves per-request workspaces out of the pool), then advances
// every active request by one macro step in lockstep: each fine and each
// coarse implicit step of the tick is one batched Newton/CG solve over all
// active requests (tl_runtime.cpp, macro_step_batch).  Requests that reach
// their macro-step count are retired: their fields, ledger and counters are
// copied to host memory and their workspace returns to the pool, so a
// request arriving while others run is admitted as soon as room frees up.
// Each request's solves use only its own buffers, scalars and partial sums,
// with its own CG launch caps, so its result does not depend on the mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "../../include/tl.h"
#include "tl_runtime_internal.h"

using namespace tl;

namespace {

// First-fit allocator over [0, size) with coalescing of freed blocks.
class PoolAllocator {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t next = it->first + bytes;
        free_.erase(it);
        if (rest) free_[next] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  std::map<size_t, size_t> free_;
};

enum ReqState { kQueued = 0, kActive = 1, kDone = 2, kFailed = 3 };

struct Request {
  uint64_t id = 0;
  tl_mesh mesh{};
  tl_material mat{};
  std::vector<tl_track> tracks;
  double t_start = 0.0;
  tl_options opts{};
  int n_macro = 0;
  size_t bytes = 0, off = 0;
  tl_sim* sim = nullptr;
  ReqState state = kQueued;
  double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;
  std::vector<double> Tc, Tf;
  int cdims[3] = {0, 0, 0}, fdims[3] = {0, 0, 0}, forigin[3] = {0, 0, 0};
  tl_stats stats{};
  tl_ledger ledger{};
  std::string err;
};

constexpr size_t kAlignS = 256;
size_t align_s(size_t x) { return (x + kAlignS - 1) / kAlignS * kAlignS; }

}  // namespace

struct tl_server {
  char* pool = nullptr;
  size_t pool_bytes = 0, budget = 0, used = 0, overhead = 0;
  int max_slots = 0;
  hipStream_t stream = nullptr;
  PoolAllocator alloc;
  std::deque<Request*> queue;
  std::vector<Request*> active;
  std::map<uint64_t, Request*> all;
  uint64_t next_id = 1;
  BatchTables tables;
  std::chrono::steady_clock::time_point t0;
  int64_t ticks = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0)
        .count();
  }
};

namespace {

tl_status sfail(tl_status st, const std::string& msg) {
  set_last_error(msg);
  return st;
}

void retire(tl_server* sv, Request* r, bool ok) {
  if (r->sim) {
    if (ok) {
      r->Tc.resize(tl_sim_nodes(r->sim, 0));
      r->Tf.resize(tl_sim_nodes(r->sim, 1));
      tl_status st = tl_get_temperature(r->sim, 0, r->Tc.data(), r->Tc.size(),
                                        r->cdims, nullptr);
      if (st == TL_OK)
        st = tl_get_temperature(r->sim, 1, r->Tf.data(), r->Tf.size(),
                                r->fdims, r->forigin);
      if (st != TL_OK) {
        ok = false;
        r->err = tl_last_error();
      }
    }
    tl_get_stats(r->sim, &r->stats);
    tl_get_ledger(r->sim, &r->ledger);
    tl_destroy(r->sim);
    r->sim = nullptr;
  }
  if (r->bytes) {
    sv->alloc.release(r->off, r->bytes);
    sv->used -= r->bytes;
  }
  r->state = ok ? kDone : kFailed;
  r->t_done = sv->now();
}

}  // namespace

extern "C" {

size_t tl_server_overhead_bytes(int max_slots) {
  if (max_slots < 1) return 0;
  return batch_tables_bytes(max_slots);
}

tl_status tl_server_create(void* dev_pool, size_t pool_bytes,
                           size_t hbm_budget, int max_slots, void* hip_stream,
                           tl_server** out) {
  if (!out) return sfail(TL_EINVAL, "out is null");
  *out = nullptr;
  if (!dev_pool || ((uintptr_t)dev_pool) % kAlignS != 0)
    return sfail(TL_EINVAL, "pool must be non-null and 256-byte aligned");
  if (max_slots < 1 || max_slots > 1024)
    return sfail(TL_EINVAL, "max_slots must be in 1..1024");
  const size_t over = align_s(batch_tables_bytes(max_slots));
  if (pool_bytes <= over)
    return sfail(TL_ENOMEM, "pool smaller than the server's own tables");
  tl_server* sv = new tl_server();
  sv->pool = (char*)dev_pool;
  sv->pool_bytes = pool_bytes;
  sv->overhead = over;
  sv->budget = std::min(hbm_budget, pool_bytes - over);
  sv->max_slots = max_slots;
  sv->stream = (hipStream_t)hip_stream;
  sv->alloc.reset(pool_bytes - over);
  sv->t0 = std::chrono::steady_clock::now();
  tl_status st = batch_tables_init(&sv->tables, sv->pool, max_slots, sv->stream);
  if (st != TL_OK) {
    delete sv;
    return st;
  }
  *out = sv;
  return TL_OK;
}

tl_status tl_server_submit(tl_server* sv, const tl_mesh* mesh,
                           const tl_material* material,
                           const tl_scan_path* scan, const tl_options* opts,
                           int n_macro, uint64_t* id) {
  if (!sv || !id) return sfail(TL_EINVAL, "null argument");
  tl_status st = validate_request(mesh, material, scan, opts);
  if (st != TL_OK) return st;
  if (n_macro < 1) return sfail(TL_EINVAL, "n_macro must be >= 1");
  const size_t bytes = align_s(tl_workspace_bytes(mesh, opts));
  if (bytes > sv->budget || bytes > sv->pool_bytes - sv->overhead)
    return sfail(TL_EBUSY, "request needs " + std::to_string(bytes) +
                               " bytes, more than the server's budget");
  Request* r = new Request();
  r->id = sv->next_id++;
  r->mesh = *mesh;
  r->mat = *material;
  r->tracks.assign(scan->tracks, scan->tracks + scan->n_tracks);
  r->t_start = scan->t_start;
  r->opts = *opts;
  r->n_macro = n_macro;
  r->bytes = bytes;
  r->t_submit = sv->now();
  sv->queue.push_back(r);
  sv->all[r->id] = r;
  *id = r->id;
  return TL_OK;
}

tl_status tl_server_tick(tl_server* sv, int* n_active, int* n_queued,
                         int* n_finished) {
  if (!sv) return sfail(TL_EINVAL, "null server");
  int finished = 0;
  // admission: arrival order, while a slot is free and the footprint fits
  while (!sv->queue.empty() && (int)sv->active.size() < sv->max_slots) {
    Request* r = sv->queue.front();
    if (sv->used + r->bytes > sv->budget) break;
    size_t off = 0;
    if (!sv->alloc.alloc(r->bytes, &off)) break;
    sv->queue.pop_front();
    r->off = off;
    sv->used += r->bytes;
    tl_scan_path sp{(int)r->tracks.size(), r->tracks.data(), r->t_start};
    tl_sim* sim = nullptr;
    tl_status st = tl_create(&r->mesh, &r->mat, &sp, &r->opts,
                             sv->pool + sv->overhead + off, r->bytes,
                             (void*)sv->stream, &sim);
    r->t_admit = sv->now();
    if (st != TL_OK) {
      r->err = tl_last_error();
      retire(sv, r, false);
      ++finished;
      continue;
    }
    r->sim = sim;
    r->state = kActive;
    sv->active.push_back(r);
  }
  // one macro step of every active request, in lockstep
  if (!sv->active.empty()) {
    std::vector<tl_sim*> sims;
    for (Request* r : sv->active) sims.push_back(r->sim);
    std::vector<std::string> errs;
    tl_status st = step_many(sims, &sv->tables, errs);
    if (st != TL_OK) return st;  // device error: the server is unusable
    std::vector<Request*> keep;
    for (size_t q = 0; q < sv->active.size(); ++q) {
      Request* r = sv->active[q];
      if (!errs[q].empty()) {
        r->err = errs[q];
        retire(sv, r, false);
        ++finished;
      } else {
        int64_t n = 0;
        tl_get_time(r->sim, nullptr, &n);
        if (n >= r->n_macro) {
          retire(sv, r, true);
          ++finished;
        } else {
          keep.push_back(r);
        }
      }
    }
    sv->active.swap(keep);
  }
  ++sv->ticks;
  if (n_active) *n_active = (int)sv->active.size();
  if (n_queued) *n_queued = (int)sv->queue.size();
  if (n_finished) *n_finished = finished;
  return TL_OK;
}

tl_status tl_server_result(tl_server* sv, uint64_t id, int level,
                           double* host_out, size_t cap, int dims_out[3],
                           tl_stats* st, tl_ledger* led,
                           tl_request_info* info) {
  if (!sv) return sfail(TL_EINVAL, "null server");
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return sfail(TL_EINVAL, "unknown request id");
  Request* r = it->second;
  if (info) {
    info->submit_s = r->t_submit;
    info->admit_s = r->t_admit;
    info->done_s = r->t_done;
    info->state = (int)r->state;
    info->macro_steps = r->state == kDone ? r->n_macro : 0;
  }
  if (r->state == kQueued || r->state == kActive)
    return sfail(TL_EBUSY, "request not finished");
  if (r->state == kFailed) return sfail(TL_ENOCONV, r->err);
  if (st) *st = r->stats;
  if (led) *led = r->ledger;
  if (host_out) {
    if (level != 0 && level != 1) return sfail(TL_EINVAL, "level must be 0 or 1");
    const std::vector<double>& v = level == 0 ? r->Tc : r->Tf;
    if (cap < v.size()) return sfail(TL_ENOMEM, "host buffer too small");
    std::memcpy(host_out, v.data(), v.size() * sizeof(double));
    if (dims_out) {
      const int* d = level == 0 ? r->cdims : r->fdims;
      dims_out[0] = d[0];
      dims_out[1] = d[1];
      dims_out[2] = d[2];
    }
  }
  return TL_OK;
}

tl_status tl_server_release(tl_server* sv, uint64_t id) {
  if (!sv) return sfail(TL_EINVAL, "null server");
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return sfail(TL_EINVAL, "unknown request id");
  Request* r = it->second;
  if (r->state == kQueued || r->state == kActive)
    return sfail(TL_EBUSY, "request not finished");
  delete r;
  sv->all.erase(it);
  return TL_OK;
}

tl_status tl_server_set_profiling(tl_server* sv, int sample_every) {
  if (!sv) return sfail(TL_EINVAL, "null server");
  return batch_set_profiling(&sv->tables, sample_every);
}

tl_status tl_server_get_profile(tl_server* sv, int64_t* launches, double* ms) {
  if (!sv) return sfail(TL_EINVAL, "null server");
  batch_get_profile(&sv->tables, launches, ms, nullptr);
  return TL_OK;
}

void tl_server_destroy(tl_server* sv) {
  if (!sv) return;
  (void)hipStreamSynchronize(sv->stream);
  for (auto& kv : sv->all) {
    Request* r = kv.second;
    if (r->sim) tl_destroy(r->sim);
    delete r;
  }
  batch_tables_free(&sv->tables);
  delete sv;
}

}  // extern "C"
