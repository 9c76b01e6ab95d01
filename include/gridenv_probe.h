/*
 * gridenv_probe.h -- a measurement tool exported by libgridenv.so beside
 * the environment API: the store pattern of the fused rollout's trajectory
 * records, with no environment work, so that the bandwidth this pattern
 * alone reaches can be set beside the fused kernel's.
 */
#ifndef GRIDENV_PROBE_H
#define GRIDENV_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Writes constant records exactly where env_rollout's fused launches of
 * k_steps steps write theirs for n_envs envs (a multiple of 64) at 64 envs
 * per tile over `blocks` persistent single-wave workgroups: for each step s
 * and tile, 64 observation records of 147 bytes (16-byte stores) at row
 * s % rows of obs [rows][n_envs][147] (16-byte aligned), then reward
 * [rows][n_envs] (float), flags and action [rows][n_envs] (bytes).  A
 * tile's 9408 observation bytes of a step leave in two pieces: aligned == 0,
 * its two 4704-byte halves; aligned != 0, as the fused kernel writes them,
 * a first piece ending on a 64-byte boundary of the output and a second one
 * with the rest.  nt != 0: non-temporal observation stores, as the fused
 * kernel's.  All buffers are caller-owned device memory of the current
 * device.  Returns 0, -1 for a bad argument (nothing launched; obs must be
 * 16-byte aligned) or -3 if the launch failed. */
int gx_probe_record_stores(uint8_t* obs, float* reward, uint8_t* flags, uint8_t* action, int64_t n_envs,
                           int32_t rows, int32_t k_steps, int32_t blocks, int32_t nt, int32_t aligned,
                           void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GRIDENV_PROBE_H */
