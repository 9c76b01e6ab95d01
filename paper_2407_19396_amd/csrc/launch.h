// launch.h -- internal interface between the host runtime (runtime.cpp) and
// the gfx950 kernels (kernels.hip).  Not part of the public C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gx {

// Per-env static tables in device memory (structure of arrays).
struct EnvTables {
  int32_t n;
  const uint32_t* meta;       // family | side << 8
  const int32_t* max_steps;   // truncation limit T >= 1
  const uint2* seed;          // Philox key (lo, hi)
  const uint32_t* rng_id;     // Philox counter word 0
  const uint64_t* grid_off;   // byte offset of the env's [S][S][3] grid
  int32_t reward_mode;        // 0: 1 - 0.9 t/T, 1: unit reward
};

// Caller-owned state (device pointers).
struct StateBufs {
  uint8_t* grid;
  int32_t *x, *y, *dir, *t, *carry;
  uint32_t* episode;
  uint8_t* done_prev;
};

// Per-step outputs: row r of each buffer holds N entries.
struct TrajBufs {
  uint8_t* obs;     // [rows][N][147] or nullptr
  float* reward;    // [rows][N]
  uint8_t* flags;   // [rows][N]
  uint8_t* action;  // [rows][N]
  int32_t rows;
};

// Fused rollout tiling: tile i covers envs [i*64, i*64+64) (the last is
// ragged); tile_cells[i] = sum of S^2 over its envs.
struct TileTables {
  int32_t n_tiles;
  int32_t max_tile_cells;     // LDS bytes of the largest tile's code grids
};

// One launch of the plain kernel: one step of every env (or the reset of
// every env when reset_all != 0).  Writes output row `row`.
hipError_t launch_plain(const EnvTables& env, const StateBufs& st, const uint8_t* actions,
                        uint64_t call, int reset_all, const TrajBufs& out, int32_t row,
                        hipStream_t stream);

// One launch of the fused kernel: k_steps steps of every env, state staged
// in LDS for the whole chunk; step s (0-based within the chunk) writes row
// (row0 + s) % rows.  actions: [k_steps][N] for this chunk, or nullptr.
hipError_t launch_fused(const EnvTables& env, const TileTables& tiles, const StateBufs& st,
                        const uint8_t* actions, uint64_t call0, int32_t k_steps,
                        const TrajBufs& out, int32_t row0, int32_t grid_blocks,
                        hipStream_t stream);

// LDS bytes one workgroup of the fused kernel needs for a tile size (static
// table and record stage plus the dynamic tile grids).
size_t fused_lds_bytes(int32_t max_tile_cells);

}  // namespace gx
