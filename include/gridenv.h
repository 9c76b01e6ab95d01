/*
 * gridenv.h -- C-ABI of libgridenv.so, an MI355X (gfx950) engine for the
 * batched gridworld environment step of NAVIX (Pignatelli et al., "NAVIX:
 * Scaling MiniGrid Environments with JAX", arXiv 2407.19396).
 *
 * The engine runs many independent MiniGrid-style environments at once
 * (Sec. 4.2 batches them with vmap; here one env per GPU lane).  One step
 * of one env is the interaction protocol of Sec. 3.2.2: the timestep
 * (t, o_t, a_t, r_{t+1}, gamma_{t+1}, s_t) is advanced by step(timestep,
 * action), which resets automatically once the episode is done; reset pads
 * the action with -1 and the reward with 0.  Inside a step the systems of
 * Table "systems" (App. A) apply in order: intervention (the action),
 * transition (identity for these families), observation, reward,
 * termination.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns 0 (GX_OK) or a negative GX_E* code and
 *   never throws.  When a call fails validation nothing is enqueued.  A
 *   fault of earlier asynchronous GPU work is reported as GX_EDEVICE by the
 *   next call that checks the device.
 * Memory: the caller allocates and frees every state, action and output
 *   buffer (device memory of the current HIP device, e.g. torch tensors).
 *   The library owns only its context (host memory plus small device
 *   tables allocated in env_create and freed in env_destroy), never frees
 *   caller memory, and allocates nothing in env_reset / env_step /
 *   env_rollout.
 * Streams: stream is a hipStream_t passed as void* (NULL = the default
 *   stream).  Calls enqueue work and return; results are valid once the
 *   stream has synchronised.  A context is not thread-safe: use it from one
 *   host thread and one stream at a time.
 * Devices: create the context with the target device current; later calls
 *   must use buffers on that device.
 *
 * Encoding (MiniGrid's canonical indices; Table "components": Tag, Colour,
 * State; Table "observations": symbolic encodings)
 *   cell triple (type, colour, state): type 0 unseen, 1 empty, 2 wall,
 *   4 door, 5 key, 8 goal; colour 0 red, 1 green, 2 blue, 3 purple,
 *   4 yellow, 5 grey; door state 0 open, 1 closed, 2 locked.
 *   Walls are (2,5,0), empty cells (1,0,0), the goal (8,1,0), keys (5,c,0),
 *   doors (4,c,s).
 *   actions: 0 turn left, 1 turn right, 2 forward, 3 pickup, 4 drop,
 *   5 toggle, 6 done; any other value acts as 6 (no effect).
 *   heading: 0 east (+x), 1 south (+y), 2 west (-x), 3 north (-y).
 *   flags bits: 1 terminated (goal reached), 2 truncated (t reached T),
 *   4 first step of an episode (reset).
 *   carry: packed triple type | colour << 8 | state << 16 of the held
 *   object; an empty hand is 1 (the triple (1,0,0)).
 *
 * State of env i (caller-owned device buffers, struct gx_state)
 *   grid: bytes [S_i][S_i][3] (row y, column x, channel) at byte offset
 *     grid_off(i) = sum_{j<i} 3 * S_j^2 of one buffer of env_sizes()
 *     bytes; the outermost ring of every grid must be walls and types
 *     must be among those listed above (every generated layout is);
 *   x, y, dir, t (int32): position, heading, steps since the last reset;
 *   carry (int32), episode (uint32: resets so far), done_prev (uint8:
 *   the last step ended the episode, so the next call resets).
 *
 * Outputs (struct gx_traj): row r of each buffer holds n_envs entries:
 *   obs: bytes [rows][n_envs][7][7][3], view row j (0 = farthest ahead,
 *     6 = the agent's row), view column i (0 = the agent's left), channel;
 *     may be NULL to skip observations;
 *   reward: float [rows][n_envs]; flags, action: bytes [rows][n_envs]
 *     (action is the action applied, 0xFF on reset steps).
 */
#ifndef GRIDENV_H
#define GRIDENV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GX_OK 0
#define GX_EINVAL -1   /* invalid argument: NULL pointer, bad size, family or side */
#define GX_ENOMEM -2   /* the context's host or device tables could not be allocated */
#define GX_EDEVICE -3  /* a HIP call failed, or earlier GPU work faulted */
#define GX_ESTATE -4   /* call order violated (e.g. a step before any reset) */

#define GX_FAMILY_EMPTY 0      /* Empty-SxS (single room), side 4..32 */
#define GX_FAMILY_TWOROOM 1    /* DoorKey-SxS (two rooms, locked door), side 5..32 */
#define GX_FAMILY_FOURROOMS 2  /* FourRooms, odd side 7..31 */

#define GX_OBS_BYTES 147

typedef struct gx_ctx gx_ctx;

/* Host description of a batch, read only during env_create. */
typedef struct {
  int32_t n_envs;              /* >= 1 */
  int32_t reward_mode;         /* 0: r = 1 - 0.9 * (t / T) on reaching the goal
                                  (Sec. 3.2.1, Eq. (1), t counted after the
                                  step, fp32); 1: r = 1 (the paper's Markovian
                                  reward) */
  const uint8_t* family;       /* [n_envs] GX_FAMILY_* */
  const uint8_t* side;         /* [n_envs] grid side S (height = width) */
  const int32_t* max_steps;    /* [n_envs] truncation limit T >= 1 */
  const uint64_t* seed;        /* [n_envs] RNG key per env, or NULL: seed_all */
  uint64_t seed_all;
  const uint32_t* rng_id;      /* [n_envs] RNG stream id per env, or NULL: i */
} gx_config;

/* Caller-owned device state (layout above). */
typedef struct {
  uint8_t* grid;
  int32_t *x, *y, *dir, *t, *carry;
  uint32_t* episode;
  uint8_t* done_prev;
} gx_state;

/* Caller-owned device outputs; `rows` rows of n_envs entries each. */
typedef struct {
  uint8_t* obs;      /* may be NULL */
  float* reward;
  uint8_t* flags;
  uint8_t* action;
  int32_t rows;      /* >= 1 */
} gx_traj;

/* Launch and tiling facts of a context (for tools and benchmarks). */
typedef struct {
  int32_t n_envs;
  int32_t n_tiles;            /* workgroup tiles of 64 envs (fused rollout) */
  int32_t max_tile_cells;     /* largest tile's cells, one LDS byte each */
  int32_t lds_bytes;          /* LDS per workgroup of the fused kernel */
  int32_t blocks;             /* persistent workgroups of the fused kernel */
  int32_t k_default;          /* steps fused per launch when K = 0 */
  uint64_t grid_bytes;
  uint64_t calls;             /* env_step calls + rollout steps since reset */
} gx_info;

/* Validate a batch description (families and sides of Table "envs"),
 * build the per-env tables (grid offsets, RNG keys) and the tiling of the
 * fused kernel, and upload them to the current device.  *out receives the
 * context, or NULL on failure. */
int env_create(const gx_config* cfg, gx_ctx** out);

/* Bytes of the grid buffer and number of envs of a context. */
int env_sizes(const gx_ctx* ctx, size_t* grid_bytes, int32_t* n_envs);

int env_info(const gx_ctx* ctx, gx_info* info);

/* reset(key) of Sec. 3.2.2 for every env: draw the start state of episode
 * 0 from the env's layout stream (Philox4x32-10 keyed by its seed, counter
 * (rng_id, episode, block, 0)), write the whole state and, when `first` is
 * not NULL, the first timestep into its row 0 (flags 4, reward 0, action
 * 0xFF).  Also restarts the context's call counter. */
int env_reset(gx_ctx* ctx, const gx_state* st, const gx_traj* first, void* stream);

/* step(timestep, action) of Sec. 3.2.2 for every env, one kernel launch:
 * envs whose previous step was done ignore their action and return the
 * first timestep of their next episode; the others apply the action and
 * return o_{t+1}, r_{t+1} and the flags.  actions: device bytes [n_envs],
 * or NULL for the uniform random policy (Philox keyed by the env seed,
 * counter (rng_id, call / 4, 1) word call % 4, call = the context's call
 * counter).  Writes output row 0 of `out`. */
int env_step(gx_ctx* ctx, const gx_state* st, const uint8_t* actions, const gx_traj* out,
             void* stream);

/* n_steps consecutive env_step calls fused into ceil(n_steps / K)
 * persistent launches that keep each env's grid in LDS and its pose in
 * registers for K steps (the jitted scan of App. B).  Step s of the call
 * writes output row s % traj->rows; the results equal n_steps env_step
 * calls bit for bit.  actions: device bytes [n_steps][n_envs] or NULL for
 * the random policy.  K = 0 picks the context's default.  No allocation
 * and no synchronisation: the call can be captured in a HIP graph. */
int env_rollout(gx_ctx* ctx, const gx_state* st, int32_t n_steps, const uint8_t* actions,
                const gx_traj* traj, int32_t K, void* stream);

/* Set the fused kernel's launch shape: steps per launch (K >= 1) and
 * persistent workgroups (blocks >= 1; 0 keeps the current value). */
int env_set_launch(gx_ctx* ctx, int32_t K, int32_t blocks);

/* Free the context and its device tables (after the stream is idle). */
int env_destroy(gx_ctx* ctx);

/* Static text for a status code. */
const char* env_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* GRIDENV_H */
