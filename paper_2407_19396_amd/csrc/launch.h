// launch.h -- internal interface between the host runtime (runtime.cpp) and
// the gfx950 kernels (kernels.hip).  Not part of the public C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gx {

// Per-env static tables in device memory (structure of arrays).
struct EnvTables {
  int32_t n;
  uint32_t* meta;             // family | side << 8 | family parameter << 16
  int32_t* max_steps;         // truncation limit T >= 1
  uint2* seed;                // Philox key (lo, hi)
  uint32_t* rng_id;           // Philox counter word 0
  uint64_t* grid_off;         // byte offset of the env's [S][S][3] grid
  int32_t reward_mode;        // 0: 1 - 0.9 t/T, 1: unit reward
  int32_t obs_mode;           // 0: symbolic first person (147 B), 1: categorical first
                              // person (49 B), 2: symbolic whole grid, 3: categorical whole grid
};

// Caller-owned state (device pointers).
struct StateBufs {
  uint8_t* grid;
  int32_t *x, *y, *dir, *t, *carry;
  uint32_t* episode;
  uint8_t* done_prev;
  uint32_t* calls;     // step calls since reset: the random policy's counter
  uint8_t* obst;       // [N][16] obstacle positions (x, y per ball, 0xFF unused)
};

// Per-step outputs: row r of each buffer holds N entries.
struct TrajBufs {
  uint8_t* obs;     // [rows][N][147], [rows][N][49], or whole-grid rows of obs_row bytes; or nullptr
  float* reward;    // [rows][N]
  uint8_t* flags;   // [rows][N]
  uint8_t* action;  // [rows][N]
  int32_t rows;
  uint64_t obs_row = 0;        // bytes of one whole-grid observation row (sum 3 S^2 or sum S^2)
  uint8_t* mission = nullptr;  // [rows][N] the episode's mission (GoToDoor colour, else 0xFF), or nullptr
};

// Fused rollout tiling: tile i covers envs [i*E, i*E+E) (the last is
// ragged), E = tile_envs envs on the first E lanes of a wave (serving: 64).
struct TileTables {
  int32_t n_tiles;
  int32_t max_tile_cells;     // LDS bytes of the largest tile's code grids (sum of S^2)
  const uint32_t* list;       // tile ids to run, n_tiles of them (serving), or nullptr: 0..n_tiles-1
  int32_t tile_envs = 64;     // E, 1..64
};

// A tile of 64 slots serving one request (device memory, 64 bytes).  The
// tile's envs are slots [tile * 64, tile * 64 + n_envs); their grids are
// contiguous from grid_base.  The record of the request's step r for its
// env l goes to index r * stride + l of its output buffers.
struct alignas(64) ServeTile {
  uint32_t active;     // 0: the tile is free
  uint32_t n_envs;     // 1..64
  uint64_t grid_base;  // byte offset of the tile's grids in the grid pool
  uint8_t* obs;        // [n_steps][stride][147] or nullptr
  float* reward;       // [n_steps][stride]
  uint8_t* flags;
  uint8_t* action;
  uint32_t stride;     // envs per output row of the request (multiple of 16)
  uint32_t local0;     // request-local index of the tile's first env
  uint32_t step0;      // steps the request has run; advanced by the kernel
  uint32_t n_steps;    // steps the request asked for
};

// Configuration of one server slot, staged in pinned host memory until the
// first launch that runs its tile copies it to the device tables.
struct SlotConfig {
  uint32_t meta;       // family | side << 8
  int32_t max_steps;
  uint2 seed;
  uint32_t rng_id;     // request-local env index
  uint32_t pad;
  uint64_t grid_off;   // byte offset of the slot's grid in the pool
};


// Whether (family, side, param) describes a valid env with side <= max_side
// (the families of Table "envs"; param: Crossings rivers, DistShift variant,
// Dynamic-Obstacles balls, KeyCorridor rows of rooms).
inline bool family_ok(int family, int side, int param, int max_side) {
  if (side > max_side || side > 32) return false;
  switch (family) {
    case 0: return side >= 4;                                  // Empty
    case 1: return side >= 5;                                  // DoorKey
    case 2: return side >= 7 && (side & 1) == 1;               // FourRooms
    case 3: return side >= 5;                                  // LavaGap
    case 4: return side >= 5 && (side & 1) == 1 && param >= 1 && param <= 8 &&
                   param <= side - 3;                          // Crossings
    case 5: return side >= 6 && (param == 1 || param == 2);    // DistShift
    case 6: return side >= 5 && param >= 1 && param <= 8 &&
                   param <= (side - 2) * (side - 2) - 2;       // Dynamic-Obstacles
    case 7: return side >= 5;                                  // GoToDoor
    case 8: return side >= 7 && (side + 2) % 3 == 0 && param >= 1 &&
                   param <= 3;                                 // KeyCorridor: side 3s - 2, R rows
    default: return false;
  }
}

// One launch of the plain kernel: one step of every env (or the reset of
// every env when reset_all != 0).  Writes output row `row`.
hipError_t launch_plain(const EnvTables& env, const StateBufs& st, const uint8_t* actions,
                        int reset_all, const TrajBufs& out, int32_t row, hipStream_t stream);

// One launch of the fused kernel: k_steps steps of every env, state staged
// in LDS for the whole chunk; step s (0-based within the chunk) writes row
// (row0 + s) % rows.  actions: [k_steps][N] for this chunk, or nullptr.
// With serve != nullptr the tiles are requests instead (see ServeTile):
// random policy, each tile runs min(k_steps, its steps left).
hipError_t launch_fused(const EnvTables& env, const TileTables& tiles, const StateBufs& st,
                        const uint8_t* actions, int32_t k_steps,
                        const TrajBufs& out, int32_t row0, int32_t grid_blocks,
                        hipStream_t stream, ServeTile* serve = nullptr,
                        const ServeTile* host_tiles = nullptr, const SlotConfig* host_slots = nullptr);

// LDS bytes one workgroup of the fused kernel needs for a tile size (static
// table and record stage plus the dynamic tile grids).
size_t fused_lds_bytes(int32_t max_tile_cells);

}  // namespace gx
