// render.h -- internal interface of the sprite renderer (render.hip) that
// turns symbolic observation records into the rgb observations of Table
// "observations" (rgb: [32H][32W][3] of the whole grid; rgb_first_person:
// [32R][32R][3] of the view).  Not part of the public C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gx {

constexpr int kSprite = 32;                            // pixels per cell side
constexpr int kSpriteBytes = kSprite * kSprite * 3;    // one [32][32][3] sprite
constexpr int kSprites = 11 * 6 * 4;                   // (type * 6 + colour) * 4 + state
constexpr int kRgbScale = kSpriteBytes / 3;            // rgb bytes per symbolic byte (1024)

// Symbolic rows written by a step kernel: obs [rows][sym_row] (first person
// [N][7][7][3], or whole grids packed like the grid buffer), and the
// scalar outputs [rows][N]; ids [rows][sym_row / 3] receives the sprite
// index of every cell (the renderer's first pass).
struct RenderSrc {
  const uint8_t* obs;
  const float* reward;
  const uint8_t* flags;
  const uint8_t* action;
  const uint8_t* mission;
  uint64_t sym_row;
  uint16_t* ids;
};

// The caller's rows: obs [rows][kRgbScale * sym_row], 16-byte aligned; the
// record of env e sits at kRgbScale times its symbolic record's offset.
// mission may be nullptr.
struct RenderDst {
  uint8_t* obs;
  float* reward;
  uint8_t* flags;
  uint8_t* action;
  uint8_t* mission;
  int32_t rows;
};

// Draw rows [0, n_rows) of src into rows (dst_row0 + r) % dst.rows of dst and
// copy their scalar outputs (two launches: sprite indices and scalars, then
// the images).  whole: records are whole grids and cell_rows lists the
// n_cell_rows (= sum of sides) cell rows of one staging row in address
// order as (index of the row's first cell among the staging row's cells,
// grid side); otherwise 7 x 7 views at 147 e, the agent's own cell drawn as
// the north-facing agent (cell_rows unused).  sprites: the device atlas
// [kSprites][32][32][3].
hipError_t launch_render(const RenderSrc& src, int32_t n_rows, int32_t n_envs, bool whole,
                         const uint2* cell_rows, uint32_t n_cell_rows, const uint8_t* sprites,
                         const RenderDst& dst, int32_t dst_row0, hipStream_t stream);

}  // namespace gx
