// render.hip -- gfx950 kernel of the rgb observation functions (Table
// "observations": rgb and rgb_first_person, 32 pixels per cell side).
//
// Every entity carries a 32 x 32 x 3 sprite (Table "components":
// HasSprite); here the sprites are an atlas in device memory, indexed by
// the cell's symbolic triple as (type * 6 + colour) * 4 + state, and the
// image of a record is its symbolic record with every cell replaced by its
// sprite.  The step kernels write symbolic records to a staging ring; this
// kernel expands them, so it is a pure stream: per env-step it reads 147
// bytes (first person) and writes 150 528.
//
// Two passes per launch of rows.  The first streams the staged records
// once: every cell's sprite index goes to a 2-byte index row (ordinary
// stores, so it stays in the caches) and the scalar outputs move to the
// caller's rows.  The staged records were just written by the step kernel's
// non-temporal stores; reading them from the draw pass, one dependent load
// at the start of every short-lived wave, cost 15 % of the draw's time.
//
// Draw pass: one 64-lane wave per piece of 2 image rows of one cell row
// (2 * 96 W contiguous bytes; 1344 B for a first-person view), pieces
// numbered in address order, a non-persistent grid.  HBM write bandwidth
// depends on the order the chip's stores arrive in: small pieces handed
// out in address order keep every compute unit's stores inside one narrow
// window sweeping the output, which measures about 25 % faster than
// workgroups that each stream a whole 150 KB image (the same bytes, more
// scattered).  Measured on 16 rows of 16 384 first-person images: pieces
// of 16, 8, 4 and 2 rows take 6.87, 6.86, 6.67 and 6.42 ms; pieces of one
// row leave 22 of 64 lanes idle and take 12.4 ms.  Lanes 0..W-1 read the
// cell row's sprite indices; each 16-byte chunk of the piece lies inside
// one sprite row of one cell, so it is one 16-byte atlas load (the atlas,
// 811 KB, stays in L2) and one non-temporal 16-byte store, two chunks per
// lane in flight.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "render.h"

namespace gx {
namespace {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int kThreads = 64;                                // one wave per piece
constexpr int kMaxSide = 32;
constexpr int kView = 7;
constexpr int kChunk = 16;
constexpr int kChunksPerSpriteRow = kSprite * 3 / kChunk;   // 6
constexpr int kPieceRows = 2;                               // image rows per piece
constexpr int kPiecesPerCellRow = kSprite / kPieceRows;     // 16
constexpr int kInFlight = 2;                                // chunks per lane per round
constexpr int kIdThreads = 256;
constexpr uint32_t kAgentCell = (kView - 1) * kView + 3;    // the agent's own cell in a view
constexpr uint32_t kAgentType = 10, kNorth = 3;

struct IdArgs {
  RenderSrc src;
  RenderDst dst;
  int32_t n;                 // envs
  int32_t dst_row0;          // caller row of staging row 0
  uint32_t cells_per_row;    // sym_row / 3
};

struct RenderArgs {
  RenderSrc src;
  RenderDst dst;
  int32_t n;                 // envs
  int32_t row0;              // first staging row of this launch
  int32_t dst_row0;          // caller row of staging row 0
  uint32_t pieces_per_row;   // first person: 7 * 16 n; whole grids: 16 * sum of sides
  uint32_t cells_per_row;    // sym_row / 3
  const uint2* crow;         // whole grids, per cell row: (index of its first cell, width)
  const uint8_t* sprites;
};

// Atlas index of a triple; a triple outside type 0..10, colour 0..5,
// state 0..3 draws sprite 0 (the unseen cell).
__device__ __forceinline__ uint32_t sprite_id(uint32_t type, uint32_t colour, uint32_t state) {
  return (type > kAgentType || colour > 5u || state > 3u) ? 0u : (type * 6u + colour) * 4u + state;
}

// Pass 1: grid (cells of a row / 256, rows).  Thread c of row r: the sprite
// index of cell c (first person: cell c % 49 of env c / 49, the agent's own
// cell drawn as the north-facing agent), and for c < n env c's scalars.
template <bool kWhole>
__global__ __launch_bounds__(kIdThreads) void k_sprite_ids(IdArgs a) {
  const uint32_t c = blockIdx.x * kIdThreads + threadIdx.x;
  const int r = (int)blockIdx.y;
  if (c >= a.cells_per_row) return;
  const uint8_t* t = a.src.obs + (uint64_t)r * a.src.sym_row + 3u * (uint64_t)c;
  uint32_t type = t[0], colour = t[1], state = t[2];
  if (!kWhole && c % (kView * kView) == kAgentCell) {
    type = kAgentType;
    colour = 0;
    state = kNorth;
  }
  a.src.ids[(uint64_t)r * a.cells_per_row + c] = (uint16_t)sprite_id(type, colour, state);
  if (c < (uint32_t)a.n) {
    const int drow = (a.dst_row0 + r) % a.dst.rows;
    const uint64_t si = (uint64_t)r * (uint64_t)a.n + c, di = (uint64_t)drow * (uint64_t)a.n + c;
    a.dst.reward[di] = a.src.reward[si];
    a.dst.flags[di] = a.src.flags[si];
    a.dst.action[di] = a.src.action[si];
    if (a.dst.mission) a.dst.mission[di] = a.src.mission[si];
  }
}

// Pass 2: the images (see the top of the file).
template <bool kWhole>
__global__ __launch_bounds__(kThreads) void k_render(RenderArgs a) {
  __shared__ uint16_t ids[kMaxSide];
  const int lane = threadIdx.x;
  const uint32_t b = blockIdx.x;
  const uint32_t rr = b / a.pieces_per_row;
  const uint32_t pc = b - rr * a.pieces_per_row;
  const int r = a.row0 + (int)rr;
  const int piece = (int)(pc & (kPiecesPerCellRow - 1));   // within the cell row
  // the cell row's first cell (its index among the row's cells) and width;
  // its image starts at kSpriteBytes times that index in the record row
  uint32_t start;
  int W;
  if (kWhole) {
    const uint2 cr = a.crow[pc / kPiecesPerCellRow];
    start = cr.x;
    W = (int)cr.y;
  } else {
    start = (pc / kPiecesPerCellRow) * kView;   // env pc / 112, cell row (pc % 112) / 16
    W = kView;
  }
  if (lane < W) ids[lane] = a.src.ids[(uint64_t)r * a.cells_per_row + start + (uint32_t)lane];
  const int drow = (a.dst_row0 + r) % a.dst.rows;
  __syncthreads();
  const int row_chunks = kChunksPerSpriteRow * W;   // 16-byte chunks per image row
  const int chunks = kPieceRows * row_chunks;
  const int py0 = piece * kPieceRows;               // first sprite row of the piece
  // q / row_chunks for q < 12 W, row_chunks = 6 W in [24, 192]: exact by
  // multiplication with floor(2^20 / row_chunks) + 1 (checked for every W)
  const uint32_t inv = (1u << 20) / (uint32_t)row_chunks + 1u;
  v4u* out = reinterpret_cast<v4u*>(a.dst.obs + (uint64_t)drow * a.src.sym_row * kRgbScale +
                                    (uint64_t)start * kSpriteBytes + (uint64_t)py0 * (uint64_t)(row_chunks * kChunk));
  const v4u* atlas = reinterpret_cast<const v4u*>(a.sprites);
  for (int q0 = 0; q0 < chunks; q0 += kInFlight * kThreads) {
    v4u v[kInFlight];
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) {
      const int q = q0 + lane + k * kThreads;
      if (q < chunks) {
        const int row = (int)(((uint32_t)q * inv) >> 20);
        const int cc = q - row * row_chunks;
        const int x = cc / kChunksPerSpriteRow;
        const int part = cc - x * kChunksPerSpriteRow;
        v[k] = atlas[(uint32_t)ids[x] * (kSpriteBytes / kChunk) +
                     (uint32_t)((py0 + row) * kChunksPerSpriteRow + part)];
      }
    }
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) {
      const int q = q0 + lane + k * kThreads;
      if (q < chunks) __builtin_nontemporal_store(v[k], out + q);
    }
  }
}

}  // namespace

hipError_t launch_render(const RenderSrc& src, int32_t n_rows, int32_t n_envs, bool whole,
                         const uint2* cell_rows, uint32_t n_cell_rows, const uint8_t* sprites,
                         const RenderDst& dst, int32_t dst_row0, hipStream_t stream) {
  if (n_rows <= 0 || n_envs <= 0) return hipSuccess;
  const uint64_t per_row = whole ? (uint64_t)kPiecesPerCellRow * n_cell_rows
                                 : (uint64_t)kView * kPiecesPerCellRow * (uint64_t)n_envs;
  if (per_row == 0 || per_row > (uint64_t)INT32_MAX) return hipErrorInvalidValue;
  // launches of as many whole rows as one grid's x dimension holds
  const uint64_t cells_per_row = src.sym_row / 3;
  if (cells_per_row > (uint64_t)UINT32_MAX - kIdThreads || n_rows > 65535) return hipErrorInvalidValue;
  {
    IdArgs ia{src, dst, n_envs, dst_row0, (uint32_t)cells_per_row};
    const dim3 grid((uint32_t)((cells_per_row + kIdThreads - 1) / kIdThreads), (uint32_t)n_rows);
    if (whole)
      hipLaunchKernelGGL(k_sprite_ids<true>, grid, dim3(kIdThreads), 0, stream, ia);
    else
      hipLaunchKernelGGL(k_sprite_ids<false>, grid, dim3(kIdThreads), 0, stream, ia);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  const int32_t rows_per_launch = (int32_t)std::max<uint64_t>(1, (uint64_t)INT32_MAX / per_row);
  for (int32_t r0 = 0; r0 < n_rows; r0 += rows_per_launch) {
    const int32_t nr = std::min(rows_per_launch, n_rows - r0);
    RenderArgs a{src, dst, n_envs, r0, dst_row0, (uint32_t)per_row, (uint32_t)cells_per_row, cell_rows, sprites};
    const dim3 grid((uint32_t)(per_row * (uint64_t)nr));
    if (whole)
      hipLaunchKernelGGL(k_render<true>, grid, dim3(kThreads), 0, stream, a);
    else
      hipLaunchKernelGGL(k_render<false>, grid, dim3(kThreads), 0, stream, a);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

}  // namespace gx
