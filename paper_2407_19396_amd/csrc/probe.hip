// probe.hip -- a measurement tool, not part of the environment step: the
// store pattern of the fused rollout kernel's trajectory records with no
// other work, to measure what that pattern alone can reach on this GPU.
//
// The launch shape and addresses are those of k_fused at 64 envs per tile:
// persistent single-wave workgroups take tiles of 64 envs in turn; for each
// step s of a chunk of k steps a tile writes its 64 observation records
// (147 bytes each, 9408 bytes in two pieces of 16-byte stores) at row s of
// the ring, then its rewards (4 bytes), flags and actions (1 byte each).
// The pieces are either the two 4704-byte halves of the block, or, as
// k_fused writes them, a first piece that ends on a 64-byte boundary of the
// output and a second one holding the rest.  The bytes written are
// constants.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gridenv_probe.h"

namespace {

constexpr int kWave = 64;
constexpr int kObs = 147;
constexpr int kHalf = 32 * kObs;          // 4704 bytes, 294 16-byte chunks

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// kNT: non-temporal observation stores.  The store kind is a template
// parameter, as in k_fused: a run-time choice between the two inside the
// store loop measured about 15 % slower than either kind alone.
template <bool kNT>
__global__ __launch_bounds__(kWave) void k_store_probe(uint8_t* obs, float* reward, uint8_t* flags,
                                                       uint8_t* action, int64_t n, int32_t rows,
                                                       int32_t k_steps, int32_t aligned) {
  const int lane = threadIdx.x;
  const int64_t n_tiles = n / kWave;
  const u32x4 v = {0x01010101u * (uint32_t)lane, 2u, 3u, 4u};
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t e0 = tile * kWave;
    for (int s = 0; s < k_steps; ++s) {
      const int64_t rec = (int64_t)(s % rows) * n;
      uint8_t* dst = obs + (rec + e0) * kObs;
      const uintptr_t d = reinterpret_cast<uintptr_t>(dst);
      // bytes of the first half that leave with the second piece
      const int keep = aligned ? (int)((d + kHalf) & 63) : 0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        u32x4* out = reinterpret_cast<u32x4*>(dst + (h ? kHalf - keep : 0));
        const int chunks = (h ? kHalf + keep : kHalf - keep) / 16;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          const int c = lane + i * kWave;
          if (c < chunks) {
            if (kNT) __builtin_nontemporal_store(v, out + c);
            else out[c] = v;
          }
        }
      }
      reward[rec + e0 + lane] = 1.0f;
      flags[rec + e0 + lane] = 1;
      action[rec + e0 + lane] = 2;
    }
  }
}

}  // namespace

extern "C" int gx_probe_record_stores(uint8_t* obs, float* reward, uint8_t* flags, uint8_t* action,
                                      int64_t n_envs, int32_t rows, int32_t k_steps, int32_t blocks,
                                      int32_t nt, int32_t aligned, void* stream) {
  if (!obs || !reward || !flags || !action || n_envs < kWave || n_envs % kWave != 0 || rows < 1 ||
      k_steps < 1 || blocks < 1 || (reinterpret_cast<uintptr_t>(obs) & 15) != 0)
    return -1;
  const auto kernel = nt ? &k_store_probe<true> : &k_store_probe<false>;
  hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kWave), 0, reinterpret_cast<hipStream_t>(stream), obs, reward,
                     flags, action, n_envs, rows, k_steps, aligned);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
