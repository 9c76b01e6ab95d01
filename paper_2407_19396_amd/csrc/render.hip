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
// One workgroup of 256 threads draws one record at a time (persistent
// over the (row, env) records of a launch).  It first turns the record's
// W x W triples into sprite ids in LDS; then thread t owns the 16-byte
// chunk t of a block of P whole image rows (an image row is 96 W bytes =
// 6 W chunks, P = floor(256 / 6W)), so each pass of the workgroup writes
// P * 96 W contiguous bytes with non-temporal 16-byte stores.  A chunk lies
// inside one sprite row of one cell, so it is one 16-byte load of the atlas
// (which stays in L2: 811 KB, the same few sprites in most cells).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "render.h"

namespace gx {
namespace {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kMaxSide = 32;
constexpr int kView = 7;
constexpr int kViewBytes = kView * kView * 3;
constexpr int kChunk = 16;
constexpr int kChunksPerSpriteRow = kSprite * 3 / kChunk;   // 6
constexpr uint32_t kAgentType = 10, kNorth = 3;

struct RenderArgs {
  RenderSrc src;
  RenderDst dst;
  int32_t n_rows, n, dst_row0;
  const uint32_t* meta;
  const uint64_t* grid_off;
  const uint8_t* sprites;
};

// Atlas index of a triple; a triple outside type 0..10, colour 0..5,
// state 0..3 draws sprite 0 (the unseen cell).
__device__ __forceinline__ uint32_t sprite_id(uint32_t type, uint32_t colour, uint32_t state) {
  return (type > kAgentType || colour > 5u || state > 3u) ? 0u : (type * 6u + colour) * 4u + state;
}

__device__ __forceinline__ v4u sprite_chunk(const uint8_t* base, const uint16_t* ids, int W, int x, int y) {
  const uint32_t id = ids[(y >> 5) * W + x];
  return *reinterpret_cast<const v4u*>(base + id * (uint32_t)kSpriteBytes + (uint32_t)(y & 31) * (kSprite * 3));
}

template <bool kWhole>
__global__ __launch_bounds__(kThreads) void k_render(RenderArgs a) {
  __shared__ uint16_t ids[kMaxSide * kMaxSide];
  const int tid = threadIdx.x;
  const int items = a.n_rows * a.n;   // < 2^31, checked by the host
  for (int it = blockIdx.x; it < items; it += gridDim.x) {
    const int r = it / a.n;
    const int e = it - r * a.n;
    const int W = kWhole ? (int)((a.meta[e] >> 8) & 0xFFu) : kView;
    const uint64_t off = kWhole ? a.grid_off[e] : (uint64_t)e * kViewBytes;
    const uint8_t* cells = a.src.obs + (uint64_t)r * a.src.sym_row + off;
    const int drow = (a.dst_row0 + r) % a.dst.rows;
    uint8_t* img = a.dst.obs + ((uint64_t)drow * a.src.sym_row + off) * kRgbScale;
    for (int c = tid; c < W * W; c += kThreads) {
      uint32_t type = cells[3 * c], colour = cells[3 * c + 1], state = cells[3 * c + 2];
      if (!kWhole && c == (kView - 1) * kView + 3) {   // the agent's own cell
        type = kAgentType;
        colour = 0;
        state = kNorth;
      }
      ids[c] = (uint16_t)sprite_id(type, colour, state);
    }
    if (tid == kThreads - 1) {
      const uint64_t si = (uint64_t)r * a.n + e, di = (uint64_t)drow * a.n + e;
      a.dst.reward[di] = a.src.reward[si];
      a.dst.flags[di] = a.src.flags[si];
      a.dst.action[di] = a.src.action[si];
      if (a.dst.mission) a.dst.mission[di] = a.src.mission[si];
    }
    __syncthreads();
    const int chunks = kChunksPerSpriteRow * W;   // per image row
    const int P = kThreads / chunks;              // image rows per pass (W <= 32: P >= 1)
    const int H = kSprite * W;
    if (tid < P * chunks) {
      const int rp = tid / chunks, cc = tid - rp * chunks;
      const int x = cc / kChunksPerSpriteRow;
      const uint8_t* base = a.sprites + (cc - kChunksPerSpriteRow * x) * kChunk;
      const uint64_t step = (uint64_t)P * (uint64_t)(chunks * kChunk);
      uint8_t* o = img + (uint64_t)rp * (uint64_t)(chunks * kChunk) + (uint64_t)cc * kChunk;
      int y = rp;
      // four rows in flight per thread: loads first, then the stores
      for (; y + 3 * P < H; y += 4 * P, o += 4 * step) {
        const v4u v0 = sprite_chunk(base, ids, W, x, y);
        const v4u v1 = sprite_chunk(base, ids, W, x, y + P);
        const v4u v2 = sprite_chunk(base, ids, W, x, y + 2 * P);
        const v4u v3 = sprite_chunk(base, ids, W, x, y + 3 * P);
        __builtin_nontemporal_store(v0, reinterpret_cast<v4u*>(o));
        __builtin_nontemporal_store(v1, reinterpret_cast<v4u*>(o + step));
        __builtin_nontemporal_store(v2, reinterpret_cast<v4u*>(o + 2 * step));
        __builtin_nontemporal_store(v3, reinterpret_cast<v4u*>(o + 3 * step));
      }
      for (; y < H; y += P, o += step)
        __builtin_nontemporal_store(sprite_chunk(base, ids, W, x, y), reinterpret_cast<v4u*>(o));
    }
    __syncthreads();   // ids are rewritten by the next record
  }
}

}  // namespace

hipError_t launch_render(const RenderSrc& src, int32_t n_rows, int32_t n_envs, bool whole,
                         const uint32_t* meta, const uint64_t* grid_off, const uint8_t* sprites,
                         const RenderDst& dst, int32_t dst_row0, int32_t blocks, hipStream_t stream) {
  if (n_rows <= 0 || n_envs <= 0) return hipSuccess;
  const int64_t items = (int64_t)n_rows * n_envs;
  if (items > INT32_MAX || blocks < 1) return hipErrorInvalidValue;
  RenderArgs a{src, dst, n_rows, n_envs, dst_row0, meta, grid_off, sprites};
  const int grid = (int)std::min<int64_t>(items, blocks);
  if (whole)
    hipLaunchKernelGGL(k_render<true>, dim3(grid), dim3(kThreads), 0, stream, a);
  else
    hipLaunchKernelGGL(k_render<false>, dim3(grid), dim3(kThreads), 0, stream, a);
  return hipGetLastError();
}

}  // namespace gx
