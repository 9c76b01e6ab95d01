// server.cpp -- continuous-batching request server of libgridenv.so.
//
// A server owns a pool of slots grouped in tiles of 64 (the fused kernel's
// unit) with their tables, state and grid storage.  A request (its own
// seed, env mix and step count) takes whole tiles; every env_server_step
// call advances all live requests by up to K steps in one persistent fused
// launch, so requests admitted while others run share the device and their
// work overlaps.  Each request's random policy counts its own steps and its
// env ids are request-local, so its results do not depend on what else is
// being served (and equal a reset + rollout of the same batch on a
// context).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <deque>
#include <new>
#include <thread>
#include <vector>

#include "../../include/gridenv.h"
#include "arena.h"
#include "launch.h"

namespace {

constexpr int kTileEnvs = 64;
constexpr int kLists = 8;   // tile lists kept for launches still in flight

struct Request {
  bool live = false;
  bool reported = false;     // its handle has been returned by env_server_step
  int32_t n_envs = 0, n_steps = 0, done = 0;
  int32_t first_tile = -1;   // its tiles, chained through gx_server::tile_next
};

}  // namespace

struct gx_server {
  int device = 0;
  int32_t max_tiles = 0, max_side = 0, reward_mode = 0;
  uint64_t tile_grid_bytes = 0, device_bytes = 0;
  // device pool
  uint32_t* d_meta = nullptr;
  int32_t* d_max_steps = nullptr;
  uint2* d_seed = nullptr;
  uint32_t* d_rng_id = nullptr;
  uint64_t* d_grid_off = nullptr;
  uint8_t* d_grid = nullptr;
  int32_t *d_x = nullptr, *d_y = nullptr, *d_dir = nullptr, *d_t = nullptr, *d_carry = nullptr;
  uint32_t* d_episode = nullptr;
  uint8_t* d_done = nullptr;
  uint32_t* d_calls = nullptr;
  uint8_t* d_obst = nullptr;
  gx::ServeTile* d_tiles = nullptr;
  // host staging of newly admitted tiles, read by their first fused launch
  // (coherent pinned memory)
  gx::ServeTile* h_tiles = nullptr;
  gx::SlotConfig* h_slots = nullptr;
  // the tile lists of the last kLists launches (read by the fused kernel
  // from coherent pinned memory); a list is reused once its launch is done
  uint32_t* h_lists = nullptr;
  hipEvent_t list_done[kLists] = {};
  int64_t launches = 0;
  // bookkeeping, sized in env_server_create so that admitting, stepping and
  // releasing allocate nothing: every live request holds at least one tile,
  // so at most max_tiles requests are live (and have handles) at once
  std::vector<int32_t> free_tiles;   // stack of free tile ids
  std::vector<int32_t> tile_next;    // the next tile of the same request, -1 after its last
  std::vector<int32_t> tile_cells;   // cells of a live tile, 0 when free
  std::vector<Request> reqs;         // by handle
  std::vector<int32_t> free_handles;
  std::vector<uint8_t> fresh;        // 1: admitted, not yet in a launch
  std::vector<int32_t> finished;     // ring of max_tiles: last step launched, handle not yet returned
  int32_t fin_head = 0, fin_count = 0;
  std::vector<int32_t> running;      // requests with steps left to launch
  int32_t live = 0;
};

namespace {

void free_all(gx_server* s) {
  void* dev[] = {s->d_meta, s->d_max_steps, s->d_seed, s->d_rng_id, s->d_grid_off, s->d_grid,
                 s->d_x, s->d_y, s->d_dir, s->d_t, s->d_carry, s->d_episode, s->d_done, s->d_calls,
                 s->d_obst, s->d_tiles};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (s->h_tiles) (void)hipHostFree(s->h_tiles);
  if (s->h_slots) (void)hipHostFree(s->h_slots);
  if (s->h_lists) (void)hipHostFree(s->h_lists);
  for (hipEvent_t& e : s->list_done)
    if (e) (void)hipEventDestroy(e);
}

template <class T>
bool dev_alloc(gx_server* s, T** p, size_t count) {
  const size_t bytes = count * sizeof(T);
  if (hipMalloc(reinterpret_cast<void**>(p), bytes) != hipSuccess) return false;
  s->device_bytes += bytes;
  return true;
}

gx::EnvTables tables_of(gx_server* s) {
  return gx::EnvTables{s->max_tiles * kTileEnvs, s->d_meta, s->d_max_steps, s->d_seed,
                       s->d_rng_id, s->d_grid_off, s->reward_mode, 0};
}

gx::StateBufs state_of(gx_server* s) {
  return gx::StateBufs{s->d_grid, s->d_x, s->d_y, s->d_dir, s->d_t, s->d_carry, s->d_episode, s->d_done,
                       s->d_calls, s->d_obst};
}

}  // namespace

extern "C" {

int env_server_create(int32_t max_tiles, int32_t max_side, int32_t reward_mode, gx_server** out) {
  if (!out) return GX_EINVAL;
  *out = nullptr;
  if (max_tiles < 1 || max_tiles > (1 << 20) || max_side < 4 || max_side > 32) return GX_EINVAL;
  if (reward_mode != 0 && reward_mode != 1) return GX_EINVAL;
  gx_server* s = new (std::nothrow) gx_server();
  if (!s) return GX_ENOMEM;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return GX_EDEVICE;
  }
  s->max_tiles = max_tiles;
  s->max_side = max_side;
  s->reward_mode = reward_mode;
  s->tile_grid_bytes = 3ull * kTileEnvs * (uint64_t)max_side * (uint64_t)max_side;
  const size_t slots = (size_t)max_tiles * kTileEnvs;
  bool ok = dev_alloc(s, &s->d_meta, slots) && dev_alloc(s, &s->d_max_steps, slots) &&
            dev_alloc(s, &s->d_seed, slots) && dev_alloc(s, &s->d_rng_id, slots) &&
            dev_alloc(s, &s->d_grid_off, slots) &&
            dev_alloc(s, &s->d_grid, (size_t)max_tiles * s->tile_grid_bytes) &&
            dev_alloc(s, &s->d_x, slots) && dev_alloc(s, &s->d_y, slots) &&
            dev_alloc(s, &s->d_dir, slots) && dev_alloc(s, &s->d_t, slots) &&
            dev_alloc(s, &s->d_carry, slots) && dev_alloc(s, &s->d_episode, slots) &&
            dev_alloc(s, &s->d_done, slots) && dev_alloc(s, &s->d_calls, slots) &&
            dev_alloc(s, &s->d_obst, slots * 16) &&
            dev_alloc(s, &s->d_tiles, (size_t)max_tiles);
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&s->h_tiles), sizeof(gx::ServeTile) * max_tiles,
                           hipHostMallocCoherent) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&s->h_slots), sizeof(gx::SlotConfig) * slots,
                           hipHostMallocCoherent) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&s->h_lists),
                           sizeof(uint32_t) * (size_t)max_tiles * kLists, hipHostMallocCoherent) == hipSuccess;
  for (hipEvent_t& e : s->list_done)
    ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  // every descriptor starts inactive
  ok = ok && hipMemset(s->d_tiles, 0, sizeof(gx::ServeTile) * max_tiles) == hipSuccess;
  if (ok) {
    try {
      // tile 0 on top of the stack: the first request takes the lowest tiles
      s->free_tiles.resize(max_tiles);
      for (int32_t t = 0; t < max_tiles; ++t) s->free_tiles[t] = max_tiles - 1 - t;
      s->tile_next.assign(max_tiles, -1);
      s->tile_cells.assign(max_tiles, 0);
      s->fresh.assign(max_tiles, 0);
      s->finished.assign(max_tiles, -1);
      s->reqs.reserve(max_tiles);
      s->free_handles.reserve(max_tiles);
      s->running.reserve(max_tiles);
    } catch (const std::bad_alloc&) {
      ok = false;
    }
  }
  if (!ok) {
    free_all(s);
    delete s;
    return GX_ENOMEM;
  }
  *out = s;
  return GX_OK;
}

int env_server_admit(gx_server* s, const gx_request* r, int32_t* handle) {
  if (!s || !r || !handle) return GX_EINVAL;
  if (r->n_envs < 1 || r->n_steps < 1 || r->stride < r->n_envs || !r->family || !r->side ||
      !r->max_steps || !r->reward || !r->flags || !r->action)
    return GX_EINVAL;
  for (int32_t i = 0; i < r->n_envs; ++i)
    if (!gx::family_ok(r->family[i], r->side[i], r->param ? r->param[i] : 0, s->max_side) ||
        r->max_steps[i] < 1)
      return GX_EINVAL;
  const int32_t need = (r->n_envs + kTileEnvs - 1) / kTileEnvs;
  if ((int32_t)s->free_tiles.size() < need) return GX_EBUSY;
  // a free tile means fewer than max_tiles live requests, so a new handle
  // stays within the capacity reserved at creation
  int32_t h;
  if (!s->free_handles.empty()) {
    h = s->free_handles.back();
    s->free_handles.pop_back();
  } else {
    h = (int32_t)s->reqs.size();
    s->reqs.emplace_back();
  }
  Request& q = s->reqs[h];
  q.live = true;
  q.reported = false;
  q.n_envs = r->n_envs;
  q.n_steps = r->n_steps;
  q.done = 0;
  q.first_tile = -1;
  const uint2 seed = make_uint2((uint32_t)r->seed, (uint32_t)(r->seed >> 32));
  int32_t prev = -1;
  for (int32_t i = 0; i < need; ++i) {
    const int32_t t = s->free_tiles.back();
    s->free_tiles.pop_back();
    s->tile_next[t] = -1;
    if (prev < 0) q.first_tile = t;
    else s->tile_next[prev] = t;
    prev = t;
    const int32_t l0 = i * kTileEnvs, n = std::min(kTileEnvs, r->n_envs - l0);
    const uint64_t base = (uint64_t)t * s->tile_grid_bytes;
    uint64_t off = base;
    int32_t cells = 0;
    for (int32_t j = 0; j < n; ++j) {
      const int32_t S = r->side[l0 + j];
      gx::SlotConfig& c = s->h_slots[(size_t)t * kTileEnvs + j];
      c.meta = (uint32_t)r->family[l0 + j] | ((uint32_t)S << 8) |
               ((uint32_t)(r->param ? r->param[l0 + j] : 0) << 16);
      c.max_steps = r->max_steps[l0 + j];
      c.seed = seed;
      c.rng_id = (uint32_t)(l0 + j);
      c.pad = 0;
      c.grid_off = off;
      off += 3ull * (uint64_t)S * (uint64_t)S;
      cells += S * S;
    }
    gx::ServeTile& d = s->h_tiles[t];
    d.active = 1;
    d.n_envs = (uint32_t)n;
    d.grid_base = base;
    d.obs = r->obs;
    d.reward = r->reward;
    d.flags = r->flags;
    d.action = r->action;
    d.stride = (uint32_t)r->stride;
    d.local0 = (uint32_t)l0;
    d.step0 = 0;
    d.n_steps = (uint32_t)r->n_steps;
    s->tile_cells[t] = cells;
    s->fresh[t] = 1;
  }
  s->live += 1;
  s->running.push_back(h);
  *handle = h;
  return GX_OK;
}

int env_server_step(gx_server* s, int32_t K, void* stream, int32_t* finished, int32_t cap,
                    int32_t* n_finished) {
  if (!s || K < 1 || cap < 0 || (cap > 0 && !finished) || !n_finished) return GX_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GX_EDEVICE;
  if (dev != s->device) return GX_EINVAL;
  if (hipGetLastError() != hipSuccess) return GX_EDEVICE;
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // launch only if some request still has steps to run: the live tiles,
  // those of requests with the most steps left first, so that the blocks
  // that finish early pick up the short ones
  if (!s->running.empty()) {
    std::sort(s->running.begin(), s->running.end(), [s](int32_t a, int32_t b) {
      const Request &qa = s->reqs[a], &qb = s->reqs[b];
      return qa.n_steps - qa.done > qb.n_steps - qb.done;
    });
    const int slot = (int)(s->launches % kLists);
    const hipError_t q = hipEventQuery(s->list_done[slot]);
    if (q == hipErrorNotReady) {
      if (hipEventSynchronize(s->list_done[slot]) != hipSuccess) return GX_EDEVICE;
    } else if (q != hipSuccess) {
      return GX_EDEVICE;
    }
    uint32_t* list = s->h_lists + (size_t)slot * s->max_tiles;
    int32_t n = 0, max_cells = 0;
    // a tile admitted since the last launch carries the top bit: that launch
    // takes its descriptor and slots from host staging and resets its envs
    for (int32_t h : s->running)
      for (int32_t t = s->reqs[h].first_tile; t >= 0; t = s->tile_next[t]) {
        list[n++] = (uint32_t)t | (s->fresh[t] ? 0x80000000u : 0u);
        s->fresh[t] = 0;
        max_cells = std::max(max_cells, s->tile_cells[t]);
      }
    // one workgroup per tile: a later tile starts on whichever workgroup
    // slot frees first, so the list (longest first) is scheduled greedily
    const int32_t blocks = n;
    const gx::TileTables tiles{n, max_cells, list};
    const gx::TrajBufs none{nullptr, nullptr, nullptr, nullptr, 1};
    if (gx::launch_fused(tables_of(s), tiles, state_of(s), nullptr, K, none, 0, blocks, st,
                         s->d_tiles, s->h_tiles, s->h_slots) != hipSuccess)
      return GX_EDEVICE;
    if (hipEventRecord(s->list_done[slot], st) != hipSuccess) return GX_EDEVICE;
    ++s->launches;
    size_t keep = 0;
    for (size_t i = 0; i < s->running.size(); ++i) {
      const int32_t h = s->running[i];
      Request& q = s->reqs[h];
      q.done += std::min(K, q.n_steps - q.done);
      if (q.done == q.n_steps) {
        // at most max_tiles handles wait here: each is live until returned
        s->finished[(s->fin_head + s->fin_count) % s->max_tiles] = h;
        ++s->fin_count;
      } else {
        s->running[keep++] = h;
      }
    }
    s->running.resize(keep);
  }
  int32_t n = 0;
  while (n < cap && s->fin_count > 0) {
    const int32_t h = s->finished[s->fin_head];
    s->reqs[h].reported = true;
    finished[n++] = h;
    s->fin_head = (s->fin_head + 1) % s->max_tiles;
    --s->fin_count;
  }
  *n_finished = n;
  return GX_OK;
}

int env_server_release(gx_server* s, int32_t handle) {
  if (!s || handle < 0 || handle >= (int32_t)s->reqs.size() || !s->reqs[handle].live) return GX_EINVAL;
  Request& q = s->reqs[handle];
  if (q.done < q.n_steps || !q.reported) return GX_ESTATE;
  for (int32_t t = q.first_tile; t >= 0;) {
    const int32_t next = s->tile_next[t];
    s->free_tiles.push_back(t);
    s->tile_cells[t] = 0;
    s->tile_next[t] = -1;
    t = next;
  }
  q.first_tile = -1;
  q.live = false;
  s->free_handles.push_back(handle);
  s->live -= 1;
  return GX_OK;
}

int env_server_info(const gx_server* s, gx_server_info* info) {
  if (!s || !info) return GX_EINVAL;
  info->max_tiles = s->max_tiles;
  info->free_tiles = (int32_t)s->free_tiles.size();
  info->live_requests = s->live;
  info->max_side = s->max_side;
  info->device_bytes = s->device_bytes;
  return GX_OK;
}

}  // extern "C"

namespace {

// A request's outputs in the arena: the scalar outputs first (one range,
// what a host delivery copies), then the observations.
struct Layout {
  uint64_t reward = 0, flags = 0, action = 0, scalars = 0, obs = 0, total = 0;
};

Layout output_layout(int32_t stride, int32_t n_steps, bool keep_obs) {
  const uint64_t recs = (uint64_t)stride * (uint64_t)n_steps;
  auto up = [](uint64_t x) { return (x + 255) & ~255ull; };
  Layout l;
  l.reward = 0;
  l.flags = up(4 * recs);
  l.action = l.flags + up(recs);
  l.scalars = l.action + up(recs);
  l.obs = l.scalars;
  l.total = l.obs + (keep_obs ? up((uint64_t)GX_OBS_BYTES * recs) : 0);
  return l;
}

// The loop of env_serve_run; its host containers may throw std::bad_alloc.
int serve_run(gx_server* s, const gx_serve_item* items, int32_t n_items, const uint8_t* family,
              const uint8_t* side, const uint8_t* param, const int32_t* max_steps, const gx_serve_opts* o,
              void* stream, double* admit_s, double* done_s, gx_serve_stats* stats) {
  if (!s || !items || n_items < 0 || !family || !side || !max_steps || !o || !admit_s || !done_s ||
      !stats || o->K < 1 || o->max_inflight < 1 || !o->arena)
    return GX_EINVAL;
  if (o->host_arena && o->host_arena_bytes < 256) return GX_EINVAL;
  if (s->live != 0) return GX_ESTATE;
  const bool deliver = o->host_arena != nullptr;
  const uint64_t budget = o->budget_bytes > s->device_bytes ? o->budget_bytes - s->device_bytes : 0;
  const uint64_t capacity = std::min<uint64_t>(o->arena_bytes, budget) & ~255ull;
  // every item must fit an idle server on its own, or the loop could wait forever
  for (int32_t i = 0; i < n_items; ++i) {
    const gx_serve_item& it = items[i];
    if (it.n_envs < 1 || it.n_steps < 1 || it.env_offset < 0 ||
        (i > 0 && it.arrival_s < items[i - 1].arrival_s))
      return GX_EINVAL;
    if ((it.n_envs + kTileEnvs - 1) / kTileEnvs > s->max_tiles) return GX_EINVAL;
    const Layout lay = output_layout((it.n_envs + 15) / 16 * 16, it.n_steps, o->keep_obs != 0);
    if (lay.total > capacity || (deliver && lay.scalars > (o->host_arena_bytes & ~255ull))) return GX_EINVAL;
  }
  using clock = std::chrono::steady_clock;
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  gx::Arena arena(capacity);
  gx::Arena host_arena(deliver ? o->host_arena_bytes : 0);
  struct Live {
    int32_t item;
    uint64_t off, bytes;     // the request's block of the device arena
    uint64_t scalars;        // bytes of its scalar outputs (the head of the block)
  };
  std::vector<Live> by_handle;
  std::vector<hipEvent_t> events(o->max_inflight + 1);
  for (auto& e : events) e = nullptr;
  // host delivery: once the host has seen a launch complete, the scalar
  // outputs of the requests it finished are copied to the host arena on a
  // stream of their own (overlapping later launches); a batch's event
  // recycles through a free list once the host has seen the copy complete
  hipStream_t copy_stream = nullptr;
  struct Copy {
    hipEvent_t ev;
    std::vector<Live> reqs;
    std::vector<uint64_t> host_off;
  };
  std::deque<Copy> copies;                       // issued, in stream order
  std::deque<std::vector<Live>> to_copy;         // waiting for host arena space
  std::vector<hipEvent_t> spare_events;
  std::deque<std::pair<int32_t, std::vector<int32_t>>> inflight;   // (event index, finished handles)
  int32_t next_event = 0;
  std::deque<int32_t> queue;
  int32_t next = 0, completed = 0, delivered = 0, launches = 0;
  uint64_t env_steps = 0;
  // every finished handle comes back from the step call that finished it
  std::vector<int32_t> fin(s->max_tiles);
  int rc = GX_OK;
  double t_admit = 0, t_step = 0, t_wait = 0;
  const auto t0 = clock::now();
  auto now_s = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
  auto take_event = [&](hipEvent_t* e) -> bool {
    if (!spare_events.empty()) {
      *e = spare_events.back();
      spare_events.pop_back();
      return true;
    }
    return hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
  };
  // issues the copies of waiting batches, in order, while host space lasts
  auto issue_copies = [&]() -> int {
    while (!to_copy.empty()) {
      std::vector<Live>& reqs = to_copy.front();
      std::vector<uint64_t> offs;
      for (const Live& l : reqs) {
        uint64_t off;
        if (!host_arena.alloc(l.scalars, &off)) {
          for (size_t k = 0; k < offs.size(); ++k) host_arena.release(offs[k], reqs[k].scalars);
          return GX_OK;   // retried when earlier copies have freed space
        }
        offs.push_back(off);
      }
      Copy c;
      if (!take_event(&c.ev)) return GX_EDEVICE;
      for (size_t k = 0; k < reqs.size(); ++k)
        if (hipMemcpyAsync(o->host_arena + offs[k], o->arena + reqs[k].off, reqs[k].scalars,
                           hipMemcpyDeviceToHost, copy_stream) != hipSuccess)
          return GX_EDEVICE;
      if (hipEventRecord(c.ev, copy_stream) != hipSuccess) return GX_EDEVICE;
      c.reqs = std::move(reqs);
      c.host_off = std::move(offs);
      copies.push_back(std::move(c));
      to_copy.pop_front();
    }
    return GX_OK;
  };
  // host side of finished copies: the results are in host memory
  auto retire_copies = [&](bool wait) -> int {
    while (!copies.empty()) {
      Copy& c = copies.front();
      const double w0 = wait ? now_s() : 0.0;
      const hipError_t q = wait ? hipEventSynchronize(c.ev) : hipEventQuery(c.ev);
      if (wait) t_wait += now_s() - w0;
      if (q == hipErrorNotReady) return GX_OK;
      if (q != hipSuccess) return GX_EDEVICE;
      const double t = now_s();
      for (size_t k = 0; k < c.reqs.size(); ++k) {
        if (o->host_done_s) o->host_done_s[c.reqs[k].item] = t;
        host_arena.release(c.host_off[k], c.reqs[k].scalars);
        arena.release(c.reqs[k].off, c.reqs[k].bytes);
        ++delivered;
      }
      spare_events.push_back(c.ev);
      copies.pop_front();
      wait = false;
    }
    return issue_copies();
  };
  // host side of finished launches, then of finished copies (polled on
  // every call, so a delivery is stamped when the host can first see it,
  // not only once the launch pipeline drains)
  auto retire = [&](bool wait) -> int {
    while (!inflight.empty()) {
      hipEvent_t ev = events[inflight.front().first];
      const double w0 = wait ? now_s() : 0.0;
      hipError_t q = wait ? hipEventSynchronize(ev) : hipEventQuery(ev);
      if (wait) t_wait += now_s() - w0;
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return GX_EDEVICE;
      const double t = now_s();
      std::vector<Live> fin_reqs;
      for (int32_t h : inflight.front().second) {
        const Live& l = by_handle[h];
        done_s[l.item] = t;
        env_steps += (uint64_t)items[l.item].n_envs * (uint64_t)items[l.item].n_steps;
        if (deliver) fin_reqs.push_back(l);
        else arena.release(l.off, l.bytes);
        if (env_server_release(s, h) != GX_OK) return GX_EDEVICE;
        ++completed;
      }
      inflight.pop_front();
      wait = false;
      if (deliver && !fin_reqs.empty()) {
        to_copy.push_back(std::move(fin_reqs));
        const int r = issue_copies();
        if (r != GX_OK) return r;
      }
    }
    return deliver ? retire_copies(false) : GX_OK;
  };
  for (auto& e : events)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = GX_EDEVICE;
  if (rc == GX_OK && deliver && hipStreamCreateWithFlags(&copy_stream, hipStreamNonBlocking) != hipSuccess)
    rc = GX_EDEVICE;
  for (int32_t i = 0; i < n_items; ++i) {
    admit_s[i] = done_s[i] = -1.0;
    if (o->host_done_s) o->host_done_s[i] = -1.0;
  }
  if (rc != GX_OK) goto out;
  while (completed < n_items || (deliver && delivered < n_items)) {
    const double t = now_s();
    while (next < n_items && items[next].arrival_s <= t) queue.push_back(next++);
    // admission in arrival order while tiles and budget allow
    const double a0 = now_s();
    while (!queue.empty()) {
      const gx_serve_item& it = items[queue.front()];
      const int32_t stride = (it.n_envs + 15) / 16 * 16;
      const Layout lay = output_layout(stride, it.n_steps, o->keep_obs != 0);
      uint64_t off;
      if (!arena.alloc(lay.total, &off)) break;
      uint8_t* base = o->arena + off;
      gx_request r;
      r.n_envs = it.n_envs;
      r.n_steps = it.n_steps;
      r.seed = it.seed;
      r.family = family + it.env_offset;
      r.side = side + it.env_offset;
      r.param = param ? param + it.env_offset : nullptr;
      r.max_steps = max_steps + it.env_offset;
      r.obs = o->keep_obs ? base + lay.obs : nullptr;
      r.reward = reinterpret_cast<float*>(base + lay.reward);
      r.flags = base + lay.flags;
      r.action = base + lay.action;
      r.stride = stride;
      int32_t h;
      const int a = env_server_admit(s, &r, &h);
      if (a == GX_EBUSY) {
        arena.release(off, lay.total);
        break;
      }
      if (a != GX_OK) {
        arena.release(off, lay.total);
        rc = a;
        goto out;
      }
      if ((int32_t)by_handle.size() <= h) by_handle.resize(h + 1);
      by_handle[h] = Live{queue.front(), off, lay.total, lay.scalars};
      admit_s[queue.front()] = t;
      queue.pop_front();
    }
    t_admit += now_s() - a0;
    // a launch only when some request still has steps to run (a request
    // whose last steps are enqueued is finished as far as launches go)
    if (!s->running.empty() && (int32_t)inflight.size() < o->max_inflight) {
      int32_t n = 0;
      const double s0 = now_s();
      rc = env_server_step(s, o->K, stream, fin.data(), (int32_t)fin.size(), &n);
      t_step += now_s() - s0;
      if (rc != GX_OK) goto out;
      if (hipEventRecord(events[next_event], st) != hipSuccess) {
        rc = GX_EDEVICE;
        goto out;
      }
      inflight.emplace_back(next_event, std::vector<int32_t>(fin.begin(), fin.begin() + n));
      next_event = (next_event + 1) % (int32_t)events.size();
      ++launches;
    }
    // wait for the oldest launch when the pipeline is full, or for the
    // oldest copy when nothing else can progress; otherwise poll
    {
      const bool full = (int32_t)inflight.size() >= o->max_inflight;
      const bool stalled = !full && inflight.empty() && s->running.empty() && !copies.empty();
      if ((rc = retire(full)) != GX_OK) goto out;
      if (stalled && (rc = retire_copies(true)) != GX_OK) goto out;
    }
    if (s->live == 0 && queue.empty() && next < n_items && copies.empty() && to_copy.empty()) {
      const double wait = items[next].arrival_s - now_s();
      if (wait > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(wait - 1e-4));
    }
  }
out:
  if (rc == GX_OK) rc = retire(true);
  if (rc == GX_OK && deliver) {
    while (rc == GX_OK && (!copies.empty() || !to_copy.empty())) rc = retire_copies(true);
  }
  if (copy_stream) (void)hipStreamSynchronize(copy_stream);
  for (auto& e : events)
    if (e) (void)hipEventDestroy(e);
  for (Copy& c : copies) (void)hipEventDestroy(c.ev);
  for (hipEvent_t e : spare_events) (void)hipEventDestroy(e);
  if (copy_stream) (void)hipStreamDestroy(copy_stream);
  stats->wall_s = now_s();
  stats->env_steps = env_steps;
  stats->completed = completed;
  stats->launches = launches;
  stats->admit_s = t_admit;
  stats->step_s = t_step;
  stats->wait_s = t_wait;
  return rc;
}

}  // namespace

extern "C" {

int env_serve_run(gx_server* s, const gx_serve_item* items, int32_t n_items, const uint8_t* family,
                  const uint8_t* side, const uint8_t* param, const int32_t* max_steps,
                  const gx_serve_opts* o, void* stream, double* admit_s, double* done_s,
                  gx_serve_stats* stats) {
  try {
    return serve_run(s, items, n_items, family, side, param, max_steps, o, stream, admit_s, done_s, stats);
  } catch (const std::bad_alloc&) {
    // launches and output copies of admitted requests may still be running
    // (on the caller's stream and the loop's copy stream): let them end
    // before the caller reuses the arenas
    (void)hipDeviceSynchronize();
    return GX_ENOMEM;
  }
}

int env_server_destroy(gx_server* s) {
  if (!s) return GX_EINVAL;
  free_all(s);
  delete s;
  return GX_OK;
}

}  // extern "C"
