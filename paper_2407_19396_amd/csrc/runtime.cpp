// runtime.cpp -- host side of libgridenv.so: argument validation, the
// per-env tables and tiling of a context, and kernel launches.  Every
// public function is extern "C", returns a GX_* status and never throws.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/gridenv.h"
#include "launch.h"
#include "render.h"

struct gx_ctx {
  int device = 0;
  int32_t n = 0;
  int32_t reward_mode = 0;
  int32_t obs_mode = 0;
  uint64_t grid_bytes = 0;
  bool has_reset = false;
  // device tables
  uint32_t* d_meta = nullptr;
  int32_t* d_max_steps = nullptr;
  uint2* d_seed = nullptr;
  uint32_t* d_rng_id = nullptr;
  uint64_t* d_grid_off = nullptr;
  // fused tiling and launch shape
  int32_t tile_envs = 64;
  int32_t n_tiles = 0;
  int32_t max_tile_cells = 0;
  int32_t blocks = 0;
  int32_t k_default = 64;
  std::vector<int32_t> cells;          // S^2 per env, for re-tiling
  // rgb modes: the sprite atlas, and the staging ring of symbolic records
  // (obs [stage_rows][sym_row], then reward, flags, action, mission
  // [stage_rows][n]) that the step kernels fill and the renderer expands
  uint8_t* d_sprites = nullptr;
  uint8_t* d_stage = nullptr;
  int32_t stage_rows = 0;
  uint2* d_cell_rows = nullptr;      // rgb whole grids: (first cell index, side) per cell row
  uint32_t n_cell_rows = 0;
};

namespace {

constexpr int kTileEnvs = 64;

// Reports (and clears) a pending asynchronous error of earlier GPU work.
int device_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GX_OK : GX_EDEVICE;
}

template <class T>
int upload(T** dst, const std::vector<T>& src) {
  if (hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(T)) != hipSuccess) return GX_ENOMEM;
  if (hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return GX_EDEVICE;
  return GX_OK;
}

void free_tables(gx_ctx* c) {
  (void)hipFree(c->d_meta);
  (void)hipFree(c->d_max_steps);
  (void)hipFree(c->d_seed);
  (void)hipFree(c->d_rng_id);
  (void)hipFree(c->d_grid_off);
  (void)hipFree(c->d_sprites);
  (void)hipFree(c->d_stage);
  (void)hipFree(c->d_cell_rows);
  c->d_sprites = nullptr;
  c->d_stage = nullptr;
  c->d_cell_rows = nullptr;
  c->d_meta = nullptr;
  c->d_max_steps = nullptr;
  c->d_seed = nullptr;
  c->d_rng_id = nullptr;
  c->d_grid_off = nullptr;
}

// Tiles of E consecutive envs, one single-wave workgroup per tile: the
// hardware starts a tile's workgroup wherever an earlier one has finished,
// which balances tiles of uneven work better than persistent workgroups
// that take their tiles in a fixed order (env_set_launch can ask for fewer).
void set_tiling(gx_ctx* c, int32_t E) {
  c->tile_envs = E;
  c->n_tiles = (c->n + E - 1) / E;
  c->max_tile_cells = 0;
  for (int32_t t = 0; t < c->n_tiles; ++t) {
    int32_t cells = 0;
    for (int32_t i = t * E; i < std::min(c->n, (t + 1) * E); ++i) cells += c->cells[i];
    c->max_tile_cells = std::max(c->max_tile_cells, cells);
  }
  c->blocks = c->n_tiles;
}

bool state_ok(const gx_state* st) {
  return st && st->grid && st->x && st->y && st->dir && st->t && st->carry && st->episode &&
         st->done_prev && st->calls && st->obst &&
         (reinterpret_cast<uintptr_t>(st->obst) & 15) == 0;
}

bool rgb_mode(const gx_ctx* c) { return c->obs_mode >= 4; }

// the observation function the step kernels compute: the rgb modes draw
// the symbolic records of the same view (4: first person, 5: whole grid)
int32_t step_obs_mode(const gx_ctx* c) {
  return c->obs_mode == 4 ? 0 : c->obs_mode == 5 ? 2 : c->obs_mode;
}

// bytes of one row of the step kernels' observation records
uint64_t sym_row_bytes(const gx_ctx* c) {
  switch (step_obs_mode(c)) {
    case 1: return (uint64_t)c->n * GX_OBS_CAT_BYTES;
    case 2: return c->grid_bytes;
    case 3: return c->grid_bytes / 3;
    default: return (uint64_t)c->n * GX_OBS_BYTES;
  }
}

// bytes of one output row of observations
uint64_t obs_row_bytes(const gx_ctx* c) {
  return rgb_mode(c) ? sym_row_bytes(c) * (uint64_t)gx::kRgbScale : sym_row_bytes(c);
}

uint64_t align256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

// staging ring layout: obs rows, then reward, flags, action, mission rows,
// then the renderer's sprite indices (2 bytes per cell)
uint64_t stage_bytes(const gx_ctx* c, int32_t rows) {
  const uint64_t n = (uint64_t)c->n;
  return align256(rows * sym_row_bytes(c)) + align256(rows * n * 4) + 3 * align256(rows * n) +
         align256(rows * (sym_row_bytes(c) / 3) * 2);
}

bool traj_ok(const gx_ctx* c, const gx_traj* tr) {
  if (!tr || !tr->reward || !tr->flags || !tr->action || tr->rows < 1) return false;
  // rgb records are written with 16-byte stores
  return !(rgb_mode(c) && tr->obs && (reinterpret_cast<uintptr_t>(tr->obs) & 15) != 0);
}

gx::EnvTables tables_of(const gx_ctx* c) {
  return gx::EnvTables{c->n, c->d_meta, c->d_max_steps, c->d_seed, c->d_rng_id, c->d_grid_off,
                       c->reward_mode, step_obs_mode(c)};
}

gx::StateBufs state_of(const gx_state* st) {
  return gx::StateBufs{st->grid, st->x, st->y, st->dir, st->t, st->carry, st->episode, st->done_prev,
                       st->calls, st->obst};
}

gx::TrajBufs traj_of(const gx_ctx* c, const gx_traj* tr) {
  return gx::TrajBufs{tr->obs, tr->reward, tr->flags, tr->action, tr->rows, sym_row_bytes(c), tr->mission};
}

// Whether the call's observations go through the staging ring (rgb modes
// with observations requested).
bool staged(const gx_ctx* c, const gx_traj* tr) { return rgb_mode(c) && tr && tr->obs; }

gx::TrajBufs stage_traj(const gx_ctx* c) {
  const uint64_t n = (uint64_t)c->n, R = (uint64_t)c->stage_rows;
  uint8_t* p = c->d_stage;
  uint8_t* obs = p;
  p += align256(R * sym_row_bytes(c));
  float* reward = reinterpret_cast<float*>(p);
  p += align256(R * n * 4);
  uint8_t* flags = p;
  p += align256(R * n);
  uint8_t* action = p;
  p += align256(R * n);
  return gx::TrajBufs{obs, reward, flags, action, c->stage_rows, sym_row_bytes(c), p};
}

uint16_t* stage_ids(const gx_ctx* c) {
  const uint64_t n = (uint64_t)c->n, R = (uint64_t)c->stage_rows;
  return reinterpret_cast<uint16_t*>(c->d_stage + align256(R * sym_row_bytes(c)) + align256(R * n * 4) +
                                     3 * align256(R * n));
}

// Draw staging rows [0, n_rows) into the caller's rows from dst_row0 on.
// When the chunk has more steps than the caller's ring has rows, its first
// n_rows - rows steps would be overwritten by later ones in the same ring
// row, so only the last tr->rows are drawn (drawing both would race).
hipError_t render_rows(const gx_ctx* c, int32_t n_rows, const gx_traj* tr, int32_t dst_row0,
                       hipStream_t stream) {
  const gx::TrajBufs s = stage_traj(c);
  const int32_t skip = std::max(0, n_rows - tr->rows);
  const uint64_t k = (uint64_t)skip, n = (uint64_t)c->n;
  const gx::RenderSrc src{s.obs + k * s.obs_row, s.reward + k * n, s.flags + k * n, s.action + k * n,
                          s.mission + k * n, s.obs_row, stage_ids(c) + k * (s.obs_row / 3)};
  const gx::RenderDst dst{tr->obs, tr->reward, tr->flags, tr->action, tr->mission, tr->rows};
  return gx::launch_render(src, n_rows - skip, c->n, c->obs_mode == 5, c->d_cell_rows, c->n_cell_rows,
                           c->d_sprites, dst, (dst_row0 + skip) % tr->rows, stream);
}

int check_device(const gx_ctx* c) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GX_EDEVICE;
  return dev == c->device ? GX_OK : GX_EINVAL;
}

}  // namespace

extern "C" {

const char* env_strerror(int status) {
  switch (status) {
    case GX_OK: return "ok";
    case GX_EINVAL: return "invalid argument";
    case GX_ENOMEM: return "out of memory";
    case GX_EDEVICE: return "HIP device error";
    case GX_ESTATE: return "call order violated (reset the envs first)";
    case GX_EBUSY: return "no free server tiles for the request now";
    case GX_ESIZE: return "batch larger than env_rollout_static's tables (GX_STATIC_MAX_ENVS envs)";
    default: return "unknown status";
  }
}

int env_create(const gx_config* cfg, gx_ctx** out) {
  if (!out) return GX_EINVAL;
  *out = nullptr;
  if (!cfg || cfg->n_envs < 1 || !cfg->family || !cfg->side || !cfg->max_steps) return GX_EINVAL;
  if (cfg->reward_mode != 0 && cfg->reward_mode != 1) return GX_EINVAL;
  if (cfg->obs_mode < 0 || cfg->obs_mode > 5) return GX_EINVAL;
  if (cfg->obs_mode >= 4 && !cfg->sprites) return GX_EINVAL;
  const int32_t n = cfg->n_envs;
  // the grid of a tile must fit the LDS of one workgroup; side <= 32 and
  // 64 envs per tile bound it at 64 KiB of cells
  std::vector<uint32_t> meta;
  std::vector<int32_t> max_steps;
  std::vector<uint2> seed;
  std::vector<uint32_t> rng_id;
  std::vector<uint64_t> grid_off;
  try {
    meta.resize(n);
    max_steps.resize(n);
    seed.resize(n);
    rng_id.resize(n);
    grid_off.resize(n);
  } catch (const std::bad_alloc&) {
    return GX_ENOMEM;
  }
  uint64_t off = 0;
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
  }
  gx_ctx* c = new (std::nothrow) gx_ctx();
  if (!c) return GX_ENOMEM;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return GX_EDEVICE;
  }
  c->n = n;
  c->reward_mode = cfg->reward_mode;
  c->obs_mode = cfg->obs_mode;
  c->grid_bytes = off;
  int rc = GX_OK;
  try {
    c->cells.resize(n);
  } catch (const std::bad_alloc&) {
    rc = GX_ENOMEM;
  }
  for (int32_t i = 0; rc == GX_OK && i < n; ++i) c->cells[i] = (int32_t)cfg->side[i] * (int32_t)cfg->side[i];
  if (rc == GX_OK) rc = upload(&c->d_meta, meta);
  if (rc == GX_OK) rc = upload(&c->d_max_steps, max_steps);
  if (rc == GX_OK) rc = upload(&c->d_seed, seed);
  if (rc == GX_OK) rc = upload(&c->d_rng_id, rng_id);
  if (rc == GX_OK) rc = upload(&c->d_grid_off, grid_off);
  if (rc == GX_OK && rgb_mode(c)) {
    // the atlas, and a staging ring of up to 64 rows within 256 MiB
    const uint64_t per_row = stage_bytes(c, 1);
    c->stage_rows = (int32_t)std::max<uint64_t>(1, std::min<uint64_t>(64, (256ull << 20) / per_row));
    try {
      const std::vector<uint8_t> atlas(cfg->sprites, cfg->sprites + (size_t)gx::kSprites * gx::kSpriteBytes);
      rc = upload(&c->d_sprites, atlas);
      if (rc == GX_OK && c->obs_mode == 5) {
        std::vector<uint2> cell_rows;
        for (int32_t i = 0; i < n; ++i)
          for (uint32_t y = 0; y < cfg->side[i]; ++y)
            cell_rows.push_back(make_uint2((uint32_t)(grid_off[i] / 3 + (uint64_t)y * cfg->side[i]), cfg->side[i]));
        c->n_cell_rows = (uint32_t)cell_rows.size();
        rc = upload(&c->d_cell_rows, cell_rows);
      }
    } catch (const std::bad_alloc&) {
      rc = GX_ENOMEM;
    }
    if (rc == GX_OK && hipMalloc(reinterpret_cast<void**>(&c->d_stage), stage_bytes(c, c->stage_rows)) !=
                           hipSuccess)
      rc = GX_ENOMEM;
  }
  if (rc != GX_OK) {
    free_tables(c);
    delete c;
    return rc;
  }
  set_tiling(c, kTileEnvs);
  *out = c;
  return GX_OK;
}

int env_sizes(const gx_ctx* c, size_t* grid_bytes, int32_t* n_envs) {
  if (!c) return GX_EINVAL;
  if (grid_bytes) *grid_bytes = (size_t)c->grid_bytes;
  if (n_envs) *n_envs = c->n;
  return GX_OK;
}

int env_info(const gx_ctx* c, gx_info* info) {
  if (!c || !info) return GX_EINVAL;
  info->n_envs = c->n;
  info->n_tiles = c->n_tiles;
  info->tile_envs = c->tile_envs;
  info->max_tile_cells = c->max_tile_cells;
  info->lds_bytes = (int32_t)gx::fused_lds_bytes(c->max_tile_cells);
  info->blocks = c->blocks;
  info->k_default = c->k_default;
  info->grid_bytes = c->grid_bytes;
  info->obs_row_bytes = obs_row_bytes(c);
  return GX_OK;
}

int env_reset(gx_ctx* c, const gx_state* st, const gx_traj* first, void* stream) {
  if (!c || !state_ok(st)) return GX_EINVAL;
  if (first && !traj_ok(c, first)) return GX_EINVAL;
  int rc = check_device(c);
  if (rc != GX_OK) return rc;
  if ((rc = device_status()) != GX_OK) return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  gx::TrajBufs tb{nullptr, nullptr, nullptr, nullptr, 1};
  if (first) tb = staged(c, first) ? stage_traj(c) : traj_of(c, first);
  if (gx::launch_plain(tables_of(c), state_of(st), nullptr, 1, tb, 0, s) != hipSuccess)
    return GX_EDEVICE;
  if (staged(c, first) && render_rows(c, 1, first, 0, s) != hipSuccess) return GX_EDEVICE;
  c->has_reset = true;
  return GX_OK;
}

int env_step(gx_ctx* c, const gx_state* st, const uint8_t* actions, const gx_traj* out,
             void* stream) {
  if (!c || !state_ok(st) || !traj_ok(c, out)) return GX_EINVAL;
  if (!c->has_reset) return GX_ESTATE;
  int rc = check_device(c);
  if (rc != GX_OK) return rc;
  if ((rc = device_status()) != GX_OK) return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool stg = staged(c, out);
  if (gx::launch_plain(tables_of(c), state_of(st), actions, 0, stg ? stage_traj(c) : traj_of(c, out), 0,
                       s) != hipSuccess)
    return GX_EDEVICE;
  if (stg && render_rows(c, 1, out, 0, s) != hipSuccess) return GX_EDEVICE;
  return GX_OK;
}

int env_rollout(gx_ctx* c, const gx_state* st, int32_t n_steps, const uint8_t* actions,
                const gx_traj* traj, int32_t K, void* stream) {
  if (!c || !state_ok(st) || !traj_ok(c, traj) || n_steps < 0 || K < 0) return GX_EINVAL;
  if (!c->has_reset) return GX_ESTATE;
  int rc = check_device(c);
  if (rc != GX_OK) return rc;
  if ((rc = device_status()) != GX_OK) return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool stg = staged(c, traj);
  // rgb: each fused launch fills the staging ring from row 0, then the
  // renderer draws those rows into the caller's ring
  const int32_t k = std::min(K > 0 ? K : c->k_default, stg ? c->stage_rows : INT32_MAX);
  const gx::TileTables tiles{c->n_tiles, c->max_tile_cells, nullptr, c->tile_envs};   // every tile, in order
  for (int32_t s0 = 0; s0 < n_steps; s0 += k) {
    const int32_t ks = std::min(k, n_steps - s0);
    const uint8_t* act = actions ? actions + (size_t)s0 * (size_t)c->n : nullptr;
    if (gx::launch_fused(tables_of(c), tiles, state_of(st), act, ks, stg ? stage_traj(c) : traj_of(c, traj),
                         stg ? 0 : s0 % traj->rows, c->blocks, s) != hipSuccess)
      return GX_EDEVICE;
    if (stg && render_rows(c, ks, traj, s0 % traj->rows, s) != hipSuccess) return GX_EDEVICE;
  }
  return GX_OK;
}

int env_set_launch(gx_ctx* c, int32_t K, int32_t blocks) {
  if (!c || K < 1 || blocks < 0) return GX_EINVAL;
  c->k_default = K;
  if (blocks > 0) c->blocks = blocks;
  return GX_OK;
}

int env_set_tiling(gx_ctx* c, int32_t tile_envs) {
  if (!c || tile_envs < 1 || tile_envs > kTileEnvs) return GX_EINVAL;
  set_tiling(c, tile_envs);
  return GX_OK;
}

int env_destroy(gx_ctx* c) {
  if (!c) return GX_EINVAL;
  free_tables(c);
  delete c;
  return GX_OK;
}

}  // extern "C"
