// static_rollout.cpp -- env_rollout_static: reset and rollout of a batch
// described by a gx_config, with the per-env tables in a file-scope device
// array instead of memory the library allocates, for callers that cannot
// allocate (code under graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  The kernels are those of env_reset and env_rollout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "../../include/gridenv.h"
#include "launch.h"

namespace {

constexpr int32_t kMaxEnvs = GX_STATIC_MAX_ENVS;
constexpr int32_t kTileEnvs = 64;
constexpr int kMaxDevices = 64;

// Table sections of the scratch array, each kMaxEnvs entries (every
// section's size is a multiple of 256 bytes, so each starts 256-aligned).
constexpr size_t kMetaOff = 0;
constexpr size_t kStepsOff = kMetaOff + sizeof(uint32_t) * kMaxEnvs;
constexpr size_t kSeedOff = kStepsOff + sizeof(int32_t) * kMaxEnvs;
constexpr size_t kRngOff = kSeedOff + sizeof(uint2) * kMaxEnvs;
constexpr size_t kOffOff = kRngOff + sizeof(uint32_t) * kMaxEnvs;
constexpr size_t kScratchBytes = kOffOff + sizeof(uint64_t) * kMaxEnvs;
static_assert(kMaxEnvs % 256 == 0, "table sections must stay 256-byte aligned");
static_assert(kScratchBytes == (size_t)GX_STATIC_MAX_ENVS * 28, "28 bytes of tables per env");

// One copy per device; host code reaches it only through the address
// hipGetSymbolAddress returns on that device.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// The host image of the tables, uploaded into the device copy by each call.
alignas(256) uint8_t g_host_tables[kScratchBytes];

// What a call needs of a device, found once per device (with it current).
struct DeviceSlot {
  uint8_t* scratch = nullptr;   // device address of scratch on this device
};

std::mutex g_mutex;                 // guards g_host_tables and g_devices
DeviceSlot g_devices[kMaxDevices];

int device_slot(int device, const DeviceSlot** out) {
  if (device < 0 || device >= kMaxDevices) return GX_EDEVICE;
  DeviceSlot& d = g_devices[device];
  if (!d.scratch) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GX_EDEVICE;
    d.scratch = static_cast<uint8_t*>(p);
  }
  *out = &d;
  return GX_OK;
}

bool state_ok(const gx_state* st) {
  return st && st->grid && st->x && st->y && st->dir && st->t && st->carry && st->episode &&
         st->done_prev && st->calls && st->obst && (reinterpret_cast<uintptr_t>(st->obst) & 15) == 0;
}

bool traj_ok(const gx_traj* tr) {
  return tr && tr->reward && tr->flags && tr->action && tr->rows >= 1;
}

}  // namespace

extern "C" int env_rollout_static(const gx_config* cfg, const gx_state* st, int32_t reset,
                                  const gx_traj* first, int32_t n_steps, const uint8_t* actions,
                                  const gx_traj* traj, int32_t K, void* stream) {
  if (!cfg || cfg->n_envs < 1 || !cfg->family || !cfg->side || !cfg->max_steps) return GX_EINVAL;
  if (cfg->n_envs > kMaxEnvs) return GX_ESIZE;
  if (cfg->reward_mode != 0 && cfg->reward_mode != 1) return GX_EINVAL;
  if (cfg->obs_mode < 0 || cfg->obs_mode > 3) return GX_EINVAL;   // no staging ring for rgb
  if (!state_ok(st) || n_steps < 0 || K < 0) return GX_EINVAL;
  if (reset && first && !traj_ok(first)) return GX_EINVAL;
  if (n_steps > 0 && !traj_ok(traj)) return GX_EINVAL;
  const int32_t n = cfg->n_envs;

  std::lock_guard<std::mutex> lock(g_mutex);
  uint32_t* meta = reinterpret_cast<uint32_t*>(g_host_tables + kMetaOff);
  int32_t* max_steps = reinterpret_cast<int32_t*>(g_host_tables + kStepsOff);
  uint2* seed = reinterpret_cast<uint2*>(g_host_tables + kSeedOff);
  uint32_t* rng_id = reinterpret_cast<uint32_t*>(g_host_tables + kRngOff);
  uint64_t* grid_off = reinterpret_cast<uint64_t*>(g_host_tables + kOffOff);
  uint64_t off = 0;
  int32_t max_tile_cells = 0, tile_cells = 0;
  for (int32_t i = 0; i < n; ++i) {
    const int fam = cfg->family[i], S = cfg->side[i], P = cfg->param ? cfg->param[i] : 0;
    if (!gx::family_ok(fam, S, P, 32) || cfg->max_steps[i] < 1) return GX_EINVAL;
    meta[i] = (uint32_t)fam | ((uint32_t)S << 8) | ((uint32_t)P << 16);
    max_steps[i] = cfg->max_steps[i];
    const uint64_t sd = cfg->seed ? cfg->seed[i] : cfg->seed_all;
    seed[i] = make_uint2((uint32_t)sd, (uint32_t)(sd >> 32));
    rng_id[i] = cfg->rng_id ? cfg->rng_id[i] : (uint32_t)i;
    grid_off[i] = off;
    off += 3ull * (uint64_t)S * (uint64_t)S;
    tile_cells += S * S;
    if ((i + 1) % kTileEnvs == 0 || i + 1 == n) {
      max_tile_cells = std::max(max_tile_cells, tile_cells);
      tile_cells = 0;
    }
  }

  int device = -1;
  if (hipGetDevice(&device) != hipSuccess) return GX_EDEVICE;
  const DeviceSlot* dev = nullptr;
  int rc = device_slot(device, &dev);
  if (rc != GX_OK) return rc;
  uint8_t* const d = dev->scratch;
  if (hipGetLastError() != hipSuccess) return GX_EDEVICE;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // the stream's earlier work (an earlier call's kernels included) reads the
  // tables before this copy replaces them; the wait makes the host image
  // free for the next call once this one returns
  const uint64_t N = (uint64_t)n;
  const struct { size_t off, bytes; } parts[] = {{kMetaOff, 4 * N}, {kStepsOff, 4 * N}, {kSeedOff, 8 * N},
                                                 {kRngOff, 4 * N}, {kOffOff, 8 * N}};
  for (const auto& p : parts)
    if (hipMemcpyAsync(d + p.off, g_host_tables + p.off, p.bytes, hipMemcpyHostToDevice, s) != hipSuccess)
      return GX_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return GX_EDEVICE;

  const int32_t obs_row_mul = cfg->obs_mode == 1 ? GX_OBS_CAT_BYTES : GX_OBS_BYTES;
  const uint64_t obs_row = cfg->obs_mode == 2 ? off : cfg->obs_mode == 3 ? off / 3 : N * obs_row_mul;
  const gx::EnvTables env{n,
                          reinterpret_cast<uint32_t*>(d + kMetaOff),
                          reinterpret_cast<int32_t*>(d + kStepsOff),
                          reinterpret_cast<uint2*>(d + kSeedOff),
                          reinterpret_cast<uint32_t*>(d + kRngOff),
                          reinterpret_cast<uint64_t*>(d + kOffOff),
                          cfg->reward_mode,
                          cfg->obs_mode};
  const gx::StateBufs sb{st->grid, st->x,       st->y,         st->dir,   st->t,
                         st->carry, st->episode, st->done_prev, st->calls, st->obst};
  if (reset) {
    gx::TrajBufs fb{nullptr, nullptr, nullptr, nullptr, 1};
    if (first) fb = gx::TrajBufs{first->obs, first->reward, first->flags, first->action, first->rows, obs_row,
                                 first->mission};
    if (gx::launch_plain(env, sb, nullptr, 1, fb, 0, s) != hipSuccess) return GX_EDEVICE;
  }
  if (n_steps == 0) return GX_OK;

  // the launch shape env_create picks: one single-wave workgroup per tile
  const int32_t n_tiles = (n + kTileEnvs - 1) / kTileEnvs;
  const int32_t blocks = n_tiles;
  const int32_t k = K > 0 ? K : 64;
  const gx::TileTables tiles{n_tiles, max_tile_cells, nullptr};
  const gx::TrajBufs tb{traj->obs, traj->reward, traj->flags, traj->action, traj->rows, obs_row, traj->mission};
  for (int32_t s0 = 0; s0 < n_steps; s0 += k) {
    const int32_t ks = std::min(k, n_steps - s0);
    const uint8_t* act = actions ? actions + (size_t)s0 * (size_t)n : nullptr;
    if (gx::launch_fused(env, tiles, sb, act, ks, tb, s0 % traj->rows, blocks, s) != hipSuccess)
      return GX_EDEVICE;
  }
  return GX_OK;
}
