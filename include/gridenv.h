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
 * transition (the identity except in Dynamic-Obstacles), observation, reward,
 * termination.  The families are those of Table "envs": Empty, DoorKey,
 * FourRooms (reward R1), the lava families LavaGap, Crossings, DistShift
 * (reward R2), Dynamic-Obstacles (reward R3), whose balls move every
 * step (its transition system), GoToDoor, whose state holds a mission, and
 * KeyCorridor (reward R1).
 * An episode terminates on reaching the goal or walking into lava (Tables
 * "rewards" and "terminations": on_goal_reached, on_lava_fall), in
 * Dynamic-Obstacles on stepping forward at a ball or wall, and in GoToDoor
 * on the done action at the mission's door (on_door_done) or on a toggle.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns 0 (GX_OK) or a negative GX_E* code and
 *   never throws.  When a call fails validation nothing is enqueued.  A
 *   fault of earlier asynchronous GPU work is reported as GX_EDEVICE by the
 *   next call that checks the device.
 * Memory: the caller allocates and frees every state, action and output
 *   buffer (device memory of the current HIP device, e.g. torch tensors).
 *   The library owns only its contexts (host memory plus small device
 *   tables allocated in env_create and freed in env_destroy) and servers
 *   (slot pools allocated in env_server_create, freed in
 *   env_server_destroy) and the fixed device array of env_rollout_static,
 *   never frees caller memory, and allocates nothing in env_reset /
 *   env_step / env_rollout / env_rollout_static / env_server_admit /
 *   env_server_step.
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
 *   4 door, 5 key, 6 ball, 8 goal, 9 lava; colour 0 red, 1 green, 2 blue,
 *   3 purple, 4 yellow, 5 grey; door state 0 open, 1 closed, 2 locked.
 *   Walls are (2,5,0), empty cells (1,0,0), the goal (8,1,0), keys (5,c,0),
 *   doors (4,c,s), lava (9,0,0), obstacles (6,2,0).
 *   actions: 0 turn left, 1 turn right, 2 forward, 3 pickup, 4 drop,
 *   5 toggle, 6 done; any other value acts as 6 (no effect).
 *   heading: 0 east (+x), 1 south (+y), 2 west (-x), 3 north (-y).
 *   flags bits: 1 terminated (goal or lava reached), 2 truncated (t reached T),
 *   4 first step of an episode (reset).
 *   carry: packed triple type | colour << 8 | state << 16 of the held
 *   object; an empty hand is 1 (the triple (1,0,0)).
 *
 * State of env i (caller-owned device buffers, struct gx_state)
 *   grid: bytes [S_i][S_i][3] (row y, column x, channel) at byte offset
 *     grid_off(i) = sum_{j<i} 3 * S_j^2 of one buffer of env_sizes()
 *     bytes; the outermost ring of every grid must be walls (GoToDoor:
 *     walls and closed doors) and types must be among those listed above
 *     (every generated layout is);
 *   x, y, dir, t (int32): position, heading, steps since the last reset;
 *   carry (int32), episode (uint32: resets so far), done_prev (uint8:
 *   the last step ended the episode, so the next call resets), calls
 *   (uint32: step calls since env_reset, the random policy's counter),
 *   obst (bytes [16] per env of family state: the Dynamic-Obstacles balls'
 *   x, y in their move order; GoToDoor's mission colour in byte 0; 0xFF in
 *   every unused byte and for the other families).
 *
 * Outputs (struct gx_traj): row r of each buffer holds n_envs entries:
 *   obs: row r is env_info's obs_row_bytes bytes; may be NULL to skip
 *     observations.  By obs_mode:
 *     0 symbolic_first_person: [n_envs][7][7][3], view row j (0 = farthest
 *       ahead, 6 = the agent's row), view column i (0 = the agent's left),
 *       channel;
 *     1 categorical_first_person: [n_envs][7][7], the type channel of 0;
 *     2 symbolic: env i's whole grid [S_i][S_i][3] at byte grid_off(i) of
 *       the row (rows are packed like the grid buffer), the agent drawn over
 *       its cell as (10, 0, heading) (MiniGrid's fully observed encoding;
 *       the carried object is not shown);
 *     3 categorical: the type channel of 2, [S_i][S_i] at grid_off(i) / 3;
 *     4 rgb_first_person: [n_envs][224][224][3], the view of mode 0 drawn
 *       with 32 x 32 sprites: pixel row 32 j + py, column 32 i + px is
 *       pixel (py, px) of view cell (i, j)'s sprite; the agent's own cell
 *       (3, 6) is drawn as the agent facing the image's top, the sprite of
 *       (10, 0, 3) (the carried object is not drawn);
 *     5 rgb: env i's whole grid of mode 2 drawn the same way,
 *       [32 S_i][32 S_i][3] at byte 1024 * grid_off(i) of the row;
 *     rows of modes 4 and 5 must start 16-byte aligned;
 *   reward: float [rows][n_envs]; flags, action: bytes [rows][n_envs]
 *     (action is the action applied, 0xFF on reset steps);
 *   mission: bytes [rows][n_envs] or NULL: the mission of the step's
 *     episode (the state's mission component, Sec. 3.2.1): GoToDoor's target
 *     door colour, 0xFF for the families without a mission.
 */
#ifndef GRIDENV_H
#define GRIDENV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GX_OK 0
#define GX_EINVAL -1   /* invalid argument: NULL pointer, bad size, family, side or param */
#define GX_ENOMEM -2   /* the context's host or device tables could not be allocated */
#define GX_EDEVICE -3  /* a HIP call failed, or earlier GPU work faulted */
#define GX_ESTATE -4   /* call order violated (e.g. a step before any reset) */
#define GX_EBUSY -5    /* a server has no free tiles for the request right now */
#define GX_ESIZE -6    /* env_rollout_static: more envs than its static tables hold */

/* Families (Table "envs").  The lava families and Dynamic-Obstacles start
 * the agent at (1, 1) facing east; walking into lava gives reward -1 in
 * both reward modes. */
#define GX_FAMILY_EMPTY 0      /* Empty-SxS (single room), side 4..32 */
#define GX_FAMILY_TWOROOM 1    /* DoorKey-SxS (two rooms, locked door), side 5..32 */
#define GX_FAMILY_FOURROOMS 2  /* FourRooms, odd side 7..31 */
#define GX_FAMILY_LAVAGAP 3    /* LavaGap-SS: a lava column with one gap, side 5..32 */
#define GX_FAMILY_CROSSINGS 4  /* Crossings-SSNN: param = N lava rivers, 1..min(8, S-3),
                                  odd side 5..31 */
#define GX_FAMILY_DISTSHIFT 5  /* DistShift: param = variant 1 or 2, side 6..32 */
#define GX_FAMILY_DYNOBS 6     /* Dynamic-Obstacles: param = balls 1..8 (at most
                                  (S-2)^2 - 2), side 5..32; three actions (any
                                  other acts as 0); every step the balls move at
                                  random first; forward at a ball or wall: -1, end */
#define GX_FAMILY_GOTODOOR 7   /* GoToDoor: a walled room of random size in the
                                  grid's top-left corner (the rest is wall), four
                                  closed doors of distinct colours, one per room
                                  wall; the mission names one colour.  done (any
                                  action >= 6) with that door directly ahead: the
                                  goal reward, end; toggle: reward 0, end.  Side
                                  5..32; no goal square */
#define GX_FAMILY_KEYCORRIDOR 8 /* KeyCorridor: param = R rows (1..3) of three
                                  rooms of size s, side = 3s - 2 (7, 10, .., 31);
                                  the middle column an open hallway, the goal
                                  behind a locked door, its key in a left room,
                                  closed doors connecting every room; the rows
                                  below the rooms are wall */

#define GX_OBS_BYTES 147      /* symbolic first-person record */
#define GX_OBS_CAT_BYTES 49   /* categorical first-person record */
#define GX_OBS_RGB_BYTES 150528 /* rgb first-person record, 224 * 224 * 3 */
#define GX_SPRITES 264          /* sprites in the atlas of the rgb modes */
#define GX_SPRITE_BYTES 3072    /* one sprite, [32][32][3] */

typedef struct gx_ctx gx_ctx;

/* Host description of a batch, read only during env_create. */
typedef struct {
  int32_t n_envs;              /* >= 1 */
  int32_t reward_mode;         /* 0: r = 1 - 0.9 * (t / T) on reaching the goal
                                  (Sec. 3.2.1, Eq. (1), t counted after the
                                  step, fp32); 1: r = 1 (the paper's Markovian
                                  reward) */
  int32_t obs_mode;            /* observation function (Table "observations"):
                                  0 symbolic_first_person, records [7][7][3]
                                  (147 bytes); 1 categorical_first_person,
                                  records [7][7] of type ids (49 bytes), the
                                  same view and occlusion; 2 symbolic, the
                                  whole grid [S][S][3]; 3 categorical, the
                                  whole grid's type ids [S][S]; 4
                                  rgb_first_person, records [224][224][3];
                                  5 rgb, the whole grid [32S][32S][3] */
  const uint8_t* family;       /* [n_envs] GX_FAMILY_* */
  const uint8_t* side;         /* [n_envs] grid side S (height = width) */
  const uint8_t* param;        /* [n_envs] family parameter, or NULL: all 0 */
  const int32_t* max_steps;    /* [n_envs] truncation limit T >= 1 */
  const uint64_t* seed;        /* [n_envs] RNG key per env, or NULL: seed_all */
  uint64_t seed_all;
  const uint32_t* rng_id;      /* [n_envs] RNG stream id per env, or NULL: i */
  const uint8_t* sprites;      /* obs_mode 4 and 5 (required there, else
                                  ignored): the sprite atlas, host bytes
                                  [264][32][32][3] copied during env_create.
                                  Every entity is drawn with the sprite of its
                                  symbolic triple (Table "components":
                                  HasSprite), sprite (type * 6 + colour) * 4 +
                                  state for type 0..10, colour 0..5, state
                                  0..3 (a door's state, the agent's heading);
                                  any other triple draws sprite 0, the unseen
                                  cell's */
} gx_config;

/* Caller-owned device state (layout above). */
typedef struct {
  uint8_t* grid;
  int32_t *x, *y, *dir, *t, *carry;
  uint32_t* episode;
  uint8_t* done_prev;
  uint32_t* calls;
  uint8_t* obst;               /* [n_envs][16], 16-byte aligned */
} gx_state;

/* Caller-owned device outputs; `rows` rows of n_envs entries each. */
typedef struct {
  uint8_t* obs;      /* may be NULL */
  float* reward;
  uint8_t* flags;
  uint8_t* action;
  int32_t rows;      /* >= 1 */
  uint8_t* mission;  /* may be NULL */
} gx_traj;

/* Launch and tiling facts of a context (for tools and benchmarks). */
typedef struct {
  int32_t n_envs;
  int32_t n_tiles;            /* workgroup tiles of tile_envs envs (fused rollout) */
  int32_t max_tile_cells;     /* largest tile's cells, one LDS byte each */
  int32_t lds_bytes;          /* LDS per workgroup of the fused kernel */
  int32_t blocks;             /* workgroups of the fused kernel (each takes tiles blocks apart) */
  int32_t k_default;          /* steps fused per launch when K = 0 */
  uint64_t grid_bytes;
  uint64_t obs_row_bytes;     /* bytes of one row of observation outputs */
  int32_t tile_envs;          /* envs per fused tile (one per lane of a wave's first lanes) */
} gx_info;

/* Validate a batch description (families and sides of Table "envs"),
 * build the per-env tables (grid offsets, RNG keys) and the tiling of the
 * fused kernel, and upload them to the current device.  In the rgb modes
 * the context also holds the sprite atlas and a staging ring of at most 64
 * rows of symbolic records (within 256 MiB, at least one row) that the
 * step kernels fill and the renderer draws; env_rollout then launches the
 * fused kernel for at most that many steps at a time, each launch followed
 * by the renderer's.  *out receives the context, or NULL on failure. */
int env_create(const gx_config* cfg, gx_ctx** out);

/* Bytes of the grid buffer and number of envs of a context. */
int env_sizes(const gx_ctx* ctx, size_t* grid_bytes, int32_t* n_envs);

int env_info(const gx_ctx* ctx, gx_info* info);

/* reset(key) of Sec. 3.2.2 for every env: draw the start state of episode
 * 0 from the env's layout stream (Philox4x32-10 keyed by its seed, counter
 * (rng_id, episode, block, 0)), write the whole state and, when `first` is
 * not NULL, the first timestep into its row 0 (flags 4, reward 0, action
 * 0xFF).  Sets every env's call counter to 0. */
int env_reset(gx_ctx* ctx, const gx_state* st, const gx_traj* first, void* stream);

/* step(timestep, action) of Sec. 3.2.2 for every env, one kernel launch:
 * envs whose previous step was done ignore their action and return the
 * first timestep of their next episode; the others apply the action and
 * return o_{t+1}, r_{t+1} and the flags.  actions: device bytes [n_envs],
 * or NULL for the uniform random policy (Philox keyed by the env seed,
 * counter (rng_id, calls / 4, 1) word calls % 4, calls = the env's step
 * calls since env_reset).  Every call, autoresetting ones included, adds 1
 * to calls.  Writes output row 0 of `out`. */
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
 * workgroups (blocks >= 1; 0 keeps the current value).  Fewer workgroups
 * than tiles are persistent: workgroup b takes tiles b, b + blocks, ...
 * The default is one workgroup per tile. */
int env_set_launch(gx_ctx* ctx, int32_t K, int32_t blocks);

/* Set the fused kernel's tiling: tiles of tile_envs (1..64, default 64)
 * consecutive envs, one env per lane on a wave's first tile_envs lanes, the
 * tile's grids in the workgroup's LDS.  Fewer envs per tile leave lanes
 * idle but need less LDS per workgroup, so more workgroups fit a compute
 * unit: the trade for large grids (Sec. 4.2 scales the batch; this picks
 * how a batch maps onto waves).  Resets the workgroup count to one per
 * tile.  Multiples of 16 keep the observation records' stores 16-byte
 * aligned; other values fall back to byte stores.  Results do not depend
 * on the tiling. */
int env_set_tiling(gx_ctx* ctx, int32_t tile_envs);

/* Free the context and its device tables (after the stream is idle). */
int env_destroy(gx_ctx* ctx);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of rollout requests.
 *
 * A server owns a pool of max_tiles tiles of 64 env slots (their tables,
 * state and grids, allocated once in env_server_create).  A request is a
 * batch of its own envs with its own seed, stepped n_steps times under the
 * random policy; it takes ceil(n_envs / 64) free tiles.  Each
 * env_server_step launch advances every live request by up to K steps, so
 * requests admitted while others run share the device.  A request's
 * results equal env_create (seed, rng_id = 0..n_envs-1) + env_reset +
 * env_rollout(n_steps, random policy) on its own envs, whatever else is
 * being served: its env ids and its policy's call counter are its own.
 * Step s of the request writes row s of its outputs (row stride `stride`
 * envs; a multiple of 16 keeps the record stores vectorised).
 * ---------------------------------------------------------------------- */
typedef struct gx_server gx_server;

typedef struct {
  int32_t n_envs;              /* >= 1 */
  int32_t n_steps;             /* >= 1 */
  uint64_t seed;               /* key of every env of the request */
  const uint8_t* family;       /* host [n_envs], read during env_server_admit */
  const uint8_t* side;         /* host [n_envs], <= the server's max_side */
  const uint8_t* param;        /* host [n_envs] family parameter, or NULL: all 0 */
  const int32_t* max_steps;    /* host [n_envs] */
  uint8_t* obs;                /* device [n_steps][stride][147], or NULL */
  float* reward;               /* device [n_steps][stride] */
  uint8_t* flags;              /* device [n_steps][stride] */
  uint8_t* action;             /* device [n_steps][stride] */
  int32_t stride;              /* >= n_envs */
} gx_request;

typedef struct {
  int32_t max_tiles, free_tiles, live_requests, max_side;
  uint64_t device_bytes;       /* device memory the server owns */
} gx_server_info;

/* Allocate a server for up to max_tiles * 64 envs of side <= max_side
 * (1 <= max_tiles <= 2^20, 4 <= max_side <= 32), with its device pool and
 * the host bookkeeping of up to max_tiles live requests, so that admitting,
 * stepping and releasing allocate nothing afterwards. */
int env_server_create(int32_t max_tiles, int32_t max_side, int32_t reward_mode, gx_server** out);

/* Queue a request (host work only; the next env_server_step's launch resets
 * its envs before their first step).  GX_EBUSY when there are not enough
 * free tiles now.
 * The output buffers must stay valid until the request is released. */
int env_server_admit(gx_server* srv, const gx_request* req, int32_t* handle);

/* Launch one fused chunk of up to K steps for every live request on
 * `stream` (newly admitted requests are reset first, in the same launch).
 * Writes to finished[0..*n_finished) the handles of requests whose last step
 * is in a launch enqueued so far (at most cap per call; the rest come with
 * later calls).  Their results are complete once the stream reaches this
 * point. */
int env_server_step(gx_server* srv, int32_t K, void* stream, int32_t* finished, int32_t cap,
                    int32_t* n_finished);

/* Return a finished request's tiles to the pool and free its handle.  Call
 * only after env_server_step has returned the handle (GX_ESTATE before) and
 * the stream has completed that request's last step. */
int env_server_release(gx_server* srv, int32_t handle);

int env_server_info(const gx_server* srv, gx_server_info* info);

/* Free the server (after its stream is idle). */
int env_server_destroy(gx_server* srv);

/* A request of a serving run: its arrival time and its envs' configuration
 * at index env_offset of the run's family / side / param / max_steps arrays
 * (param may be NULL: all 0). */
typedef struct {
  double arrival_s;            /* seconds from the start of the run, non-decreasing */
  int32_t n_envs, n_steps;
  uint64_t seed;
  int64_t env_offset;
} gx_serve_item;

typedef struct {
  int32_t K;                   /* steps per launch */
  int32_t max_inflight;        /* launches enqueued ahead of the device */
  int32_t keep_obs;            /* 1: requests get observation outputs */
  uint64_t budget_bytes;       /* HBM budget: the server's pool plus request outputs */
  uint8_t* arena;              /* device memory for request outputs */
  uint64_t arena_bytes;
  uint8_t* host_arena;         /* pinned host memory (hipHostMalloc) to deliver each request's
                                  scalar outputs to, or NULL: results stay in HBM */
  uint64_t host_arena_bytes;
  double* host_done_s;         /* [n_items] out, or NULL: when a request's scalar outputs
                                  were in host_arena (seconds from the start; -1 if not) */
} gx_serve_opts;

typedef struct {
  double wall_s;               /* run time */
  uint64_t env_steps;          /* env-steps of completed requests */
  int32_t completed, launches;
  double admit_s;              /* host time spent admitting requests */
  double step_s;               /* host time spent enqueuing launches */
  double wait_s;               /* host time blocked on the device */
} gx_serve_stats;

/* Serve items in real time on an idle server: admit each request when it
 * has arrived, in arrival order, once tiles free up and its outputs fit the
 * budget (outputs are carved from the arena, row stride rounded up to 16
 * envs: reward, flags and action first, then the observations); step every
 * live request K steps per launch with up to max_inflight launches ahead of
 * the device (a launch only while some request has steps left); a request
 * completes on the device when the host sees its last launch finish, and
 * its tiles are then reused.  With a host arena its scalar outputs (reward,
 * flags, action: 6 bytes per env-step plus padding) are then copied there
 * on a stream of the library's own, and its device outputs are reused once
 * that copy has finished; the observations stay in HBM for an on-device
 * consumer.  The host arena's contents are overwritten by later requests.
 * admit_s / done_s [n_items] receive admission and device-completion times
 * (seconds from the start); latency = done_s - arrival_s, or
 * host_done_s - arrival_s to the host.  EINVAL when a request alone would
 * not fit the arenas. */
int env_serve_run(gx_server* srv, const gx_serve_item* items, int32_t n_items,
                  const uint8_t* family, const uint8_t* side, const uint8_t* param,
                  const int32_t* max_steps, const gx_serve_opts* opts, void* stream,
                  double* admit_s, double* done_s,
                  gx_serve_stats* stats);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 *
 * env_rollout_static runs what env_create(cfg), then env_reset(st, first)
 * when reset != 0, then env_rollout(st, n_steps, actions, traj, K) and
 * env_destroy would run, with bit-identical results, but allocates nothing:
 * the per-env tables (28 bytes per env) live in a fixed array of the
 * library's device code, GX_STATIC_MAX_ENVS envs' worth (7 MiB), which
 * each device the library runs on holds until the process ends.  Launch
 * shape: env_create's workgroup count; K = 0 means 64 steps per launch.
 * Observation modes 0..3 only (EINVAL for the rgb modes, whose staging ring
 * would not be modest); GX_ESIZE when cfg->n_envs > GX_STATIC_MAX_ENVS.
 * With reset == 0 the state must come from an earlier reset of the same
 * batch description (by either entry point); first may be NULL.
 * The call uploads the tables on `stream` and waits for that upload (and so
 * for the stream's earlier work) before it enqueues the kernels: it cannot
 * be captured in a graph, and it returns with the kernels still running.
 * Every call on one device shares that device's tables: calls that overlap
 * on one device (other streams or host threads whose kernels are still
 * running) race; host threads are serialised only while they upload. */
#define GX_STATIC_MAX_ENVS 262144
int env_rollout_static(const gx_config* cfg, const gx_state* st, int32_t reset, const gx_traj* first,
                       int32_t n_steps, const uint8_t* actions, const gx_traj* traj, int32_t K,
                       void* stream);

/* Static text for a status code. */
const char* env_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* GRIDENV_H */
