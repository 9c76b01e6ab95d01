// kernels.hip -- gfx950 kernels of the batched gridworld environment step.
//
// The step is NAVIX's interaction protocol (arXiv 2407.19396, Sec. 3.2.2:
// step(timestep, action) with autoreset; reset pads action -1, reward 0)
// applied to MiniGrid's dynamics, which the paper reproduces exactly
// (Sec. 3.2.1): the intervention / transition / observation / reward /
// termination systems of Table "systems" and App. A over the Wall, Key,
// Door and Goal entities of Table "entities".
//
// Two kernels share the device functions below:
//   k_plain  -- one launch per step; one env per lane; state, grid and
//               outputs in HBM; view cells read straight from the grid.
//   k_fused  -- persistent; each workgroup takes tiles of 64 envs of any
//               mix of sizes, stages their grids in LDS as one byte per
//               cell, runs K steps with the pose in registers, writes one
//               trajectory record per env-step, then writes the state back.
// Both stage the 147-byte observations of a wave through LDS so that the
// wave's 64 records leave as one contiguous, 16-byte-vectorised block.
//
// All arithmetic is integer except the reward, which is three separately
// rounded fp32 operations (built with -ffp-contract=off).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"

namespace gx {
namespace {

constexpr int kWave = 64;
constexpr int kView = 7;
constexpr int kObsBytes = kView * kView * 3;        // 147
constexpr int kStageBytes = kWave * kObsBytes;      // 9408, a multiple of 16
constexpr int kObsWords = 37;                       // ceil(147 / 4)

// Cell triples are packed as type | colour << 8 | state << 16 (MiniGrid's
// object, colour and state indices).  Bit 31 marks a see-through cell.
constexpr uint32_t kEmpty = 1, kWall = 2, kDoor = 4, kKey = 5, kBall = 6, kBox = 7, kGoal = 8;
constexpr uint32_t kGreen = 1, kGrey = 5;
constexpr uint32_t kOpen = 0, kClosed = 1, kLocked = 2;
constexpr uint32_t kSeeBit = 1u << 31;
constexpr uint32_t kCellWall = kWall | (kGrey << 8);
constexpr uint32_t kCellEmpty = kEmpty;
constexpr uint32_t kCellGoal = kGoal | (kGreen << 8);

constexpr uint32_t kFlagTerminated = 1, kFlagTruncated = 2, kFlagFirst = 4;
constexpr uint32_t kActionNone = 0xFF;

enum : uint32_t { kLeft = 0, kRight = 1, kForward = 2, kPickup = 3, kDrop = 4, kToggle = 5 };
enum : uint32_t { kFamEmpty = 0, kFamTwoRoom = 1, kFamFourRooms = 2 };

__device__ __forceinline__ uint32_t see_through(uint32_t tri) {
  const uint32_t type = tri & 0xFF, state = (tri >> 16) & 0xFF;
  const bool opaque = type == kWall || (type == kDoor && state != kOpen);
  return opaque ? 0u : kSeeBit;
}

// heading d: 0 east (+x), 1 south (+y), 2 west, 3 north
__device__ __forceinline__ int dir_dx(int d) { return (d & 1) ? 0 : 1 - d; }
__device__ __forceinline__ int dir_dy(int d) { return (d & 1) ? 2 - d : 0; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): counter-based, so every draw is a
// pure function of (key, counter) and needs no stored generator state.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

// uniform integer in [0, n)
__device__ __forceinline__ uint32_t bounded(uint32_t word, uint32_t n) { return __umulhi(word, n); }

__device__ __forceinline__ uint32_t pick4(uint4 v, uint32_t lane) {
  uint32_t r = v.x;
  r = lane == 1 ? v.y : r;
  r = lane == 2 ? v.z : r;
  r = lane == 3 ? v.w : r;
  return r;
}

// Random-policy words for call block `call >> 2`: counter (id, block lo, block hi, 1).
__device__ __forceinline__ uint4 policy_block(uint2 seed, uint32_t rng_id, uint64_t call) {
  const uint64_t blk = call >> 2;
  return philox10(make_uint4(rng_id, (uint32_t)blk, (uint32_t)(blk >> 32), 1u), seed);
}

// ---------------------------------------------------------------------------
// Start states (reset(key) of Sec. 3.2.2; the families of Table "envs").
// Layout parameters come from the layout stream, counter (id, episode,
// block, 0), in draw order; "uniform placement" picks the k-th free cell
// in row-major order, which every family below reaches in closed form.
// ---------------------------------------------------------------------------
struct Layout {
  int fam, S;
  int a, b, c, d;      // TwoRoom: a = wall column, b = door row; FourRooms: the 4 openings
  int colour;          // TwoRoom door / key colour
  int kx, ky;          // TwoRoom key
  int gx, gy;          // goal
  int ax, ay, dir;     // agent
};

__device__ __forceinline__ void fourrooms_cell(int S, int m, int g1, int g2, int g3, int g4,
                                               uint32_t idx, int& x, int& y) {
  // idx-th free cell, row-major, of a four-room grid with openings
  // (m, g1), (m, g2) in the vertical wall and (g3, m), (g4, m) in the horizontal one
  y = 1;
  for (int yy = 1; yy <= S - 2; ++yy) {
    const uint32_t cnt = yy == m ? 2u : (uint32_t)(S - 2) - ((yy == g1 || yy == g2) ? 0u : 1u);
    if (idx < cnt) {
      y = yy;
      if (yy == m) {
        x = idx == 0 ? g3 : g4;
      } else if (yy == g1 || yy == g2) {
        x = 1 + (int)idx;
      } else {
        x = 1 + (int)idx;
        if (x >= m) x += 1;
      }
      return;
    }
    idx -= cnt;
  }
  x = 1;
}

__device__ Layout make_layout(uint32_t fam, int S, uint2 seed, uint32_t rng_id, uint32_t episode) {
  const uint4 w0 = philox10(make_uint4(rng_id, episode, 0u, 0u), seed);
  const uint4 w1 = philox10(make_uint4(rng_id, episode, 1u, 0u), seed);
  Layout L;
  L.fam = (int)fam;
  L.S = S;
  L.a = L.b = L.c = L.d = -1;
  L.colour = 0;
  L.kx = L.ky = -1;
  L.gx = S - 2;
  L.gy = S - 2;
  if (fam == kFamEmpty) {
    const int w = S - 2;
    const uint32_t k = bounded(w0.x, (uint32_t)(w * w - 1));   // interior minus the last (goal) cell
    L.ax = 1 + (int)(k % (uint32_t)w);
    L.ay = 1 + (int)(k / (uint32_t)w);
    L.dir = (int)bounded(w0.y, 4u);
  } else if (fam == kFamTwoRoom) {
    L.a = 2 + (int)bounded(w0.x, (uint32_t)(S - 4));
    L.b = 1 + (int)bounded(w0.y, (uint32_t)(S - 3));
    L.colour = (int)bounded(w0.z, 6u);
    const uint32_t lw = (uint32_t)(L.a - 1), n = lw * (uint32_t)(S - 2);
    const uint32_t kk = bounded(w0.w, n);
    L.kx = 1 + (int)(kk % lw);
    L.ky = 1 + (int)(kk / lw);
    uint32_t ka = bounded(w1.x, n - 1u);
    ka += ka >= kk ? 1u : 0u;
    L.ax = 1 + (int)(ka % lw);
    L.ay = 1 + (int)(ka / lw);
    L.dir = (int)bounded(w1.y, 4u);
  } else {
    const int m = S / 2;
    L.a = 1 + (int)bounded(w0.x, (uint32_t)(m - 1));
    L.b = m + 1 + (int)bounded(w0.y, (uint32_t)(m - 1));
    L.c = 1 + (int)bounded(w0.z, (uint32_t)(m - 1));
    L.d = m + 1 + (int)bounded(w0.w, (uint32_t)(m - 1));
    const uint32_t nfree = (uint32_t)((S - 2) * (S - 2)) - (uint32_t)(2 * (S - 2) - 1) + 4u;
    const uint32_t kg = bounded(w1.x, nfree);
    fourrooms_cell(S, m, L.a, L.b, L.c, L.d, kg, L.gx, L.gy);
    uint32_t ka = bounded(w1.y, nfree - 1u);
    ka += ka >= kg ? 1u : 0u;
    fourrooms_cell(S, m, L.a, L.b, L.c, L.d, ka, L.ax, L.ay);
    L.dir = (int)bounded(w1.z, 4u);
  }
  return L;
}

// content of cell (x, y) of a freshly generated layout (triple, no see bit)
__device__ __forceinline__ uint32_t layout_cell(const Layout& L, int x, int y) {
  const int S = L.S;
  if (x == 0 || y == 0 || x == S - 1 || y == S - 1) return kCellWall;
  if (x == L.gx && y == L.gy) return kCellGoal;
  if (L.fam == kFamTwoRoom) {
    if (x == L.a) return y == L.b ? (kDoor | ((uint32_t)L.colour << 8) | (kLocked << 16)) : kCellWall;
    if (x == L.kx && y == L.ky) return kKey | ((uint32_t)L.colour << 8);
  } else if (L.fam == kFamFourRooms) {
    const int m = S / 2;
    if (x == m) return (y == L.a || y == L.b) ? kCellEmpty : kCellWall;
    if (y == m) return (x == L.c || x == L.d) ? kCellEmpty : kCellWall;
  }
  return kCellEmpty;
}

__device__ __forceinline__ int bcast(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

__device__ __forceinline__ Layout bcast_layout(const Layout& L, int r) {
  Layout o;
  o.fam = bcast(L.fam, r); o.S = bcast(L.S, r);
  o.a = bcast(L.a, r); o.b = bcast(L.b, r); o.c = bcast(L.c, r); o.d = bcast(L.d, r);
  o.colour = bcast(L.colour, r);
  o.kx = bcast(L.kx, r); o.ky = bcast(L.ky, r);
  o.gx = bcast(L.gx, r); o.gy = bcast(L.gy, r);
  o.ax = o.ay = o.dir = 0;
  return o;
}

// ---------------------------------------------------------------------------
// Intervention I(s, a) (Table "systems"; App. A): turn, forward with
// collision, pickup, drop, toggle.  `front` is the triple ahead.
// ---------------------------------------------------------------------------
struct ActResult {
  uint32_t new_front;
  bool front_changed;
  bool terminated;
};

__device__ __forceinline__ ActResult intervene(uint32_t act, int& x, int& y, int& dir, uint32_t& carry,
                                               uint32_t front, int fx, int fy) {
  const uint32_t type = front & 0xFF, colour = (front >> 8) & 0xFF, state = (front >> 16) & 0xFF;
  ActResult r{front & 0xFFFFFFu, false, false};
  if (act == kLeft) {
    dir = (dir + 3) & 3;
  } else if (act == kRight) {
    dir = (dir + 1) & 3;
  } else if (act == kForward) {
    const bool walk = type == kEmpty || type == kGoal || (type == kDoor && state == kOpen);
    if (walk) {
      x = fx;
      y = fy;
    }
    r.terminated = type == kGoal;
  } else if (act == kPickup) {
    if (carry == kCellEmpty && (type == kKey || type == kBall || type == kBox)) {
      carry = front & 0xFFFFFFu;
      r.new_front = kCellEmpty;
      r.front_changed = true;
    }
  } else if (act == kDrop) {
    if (carry != kCellEmpty && type == kEmpty) {
      r.new_front = carry;
      carry = kCellEmpty;
      r.front_changed = true;
    }
  } else if (act == kToggle) {
    if (type == kDoor) {
      if (state == kLocked) {
        if ((carry & 0xFF) == kKey && ((carry >> 8) & 0xFF) == colour) {
          r.new_front = kDoor | (colour << 8) | (kOpen << 16);
          r.front_changed = true;
        }
      } else {
        r.new_front = kDoor | (colour << 8) | ((state == kOpen ? kClosed : kOpen) << 16);
        r.front_changed = true;
      }
    }
  }
  return r;
}

// Reward of Eq. (1) in the time-discounted form 1 - 0.9 * (t / T), t after
// the step, as three IEEE fp32 operations; reward_mode 1: unit reward.
__device__ __forceinline__ float goal_reward(int32_t t, int32_t T, int32_t mode) {
  if (mode == 1) return 1.0f;
  const float q = __fdiv_rn((float)t, (float)T);
  const float p = __fmul_rn(0.9f, q);
  return __fsub_rn(1.0f, p);
}

// ---------------------------------------------------------------------------
// Observation O(s) (Table "observations", symbolic_first_person, R = 7):
// the 7x7 view ahead of the agent, agent at view column 3 of row 6; walls
// and non-open doors block sight.  Per view row the visible cells are the
// seeds plus the see-through runs that touch a see-through seed, widened
// by one cell on each side; the next row's seeds are the three cells ahead
// of every visible see-through cell.  This is MiniGrid's two-pass rule in
// bit-parallel form: the run fills are carry propagations, the downward
// one in bit-reversed space.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t visible_row(uint32_t seeds, uint32_t see, uint32_t& next) {
  const uint32_t g = seeds & see;
  const uint32_t up = (((see + g) ^ see) | g) & see;
  const uint32_t rs = __builtin_bitreverse32(see), rg = __builtin_bitreverse32(g);
  const uint32_t down = __builtin_bitreverse32((((rs + rg) ^ rs) | rg) & rs);
  const uint32_t run = up | down;
  next = (run | (run << 1) | (run >> 1)) & 0x7Fu;
  return seeds | next;
}

// Fills w[37] with the 147-byte record obs[j][i][c].  Cells(x, y) returns
// the triple of world cell (x, y) with kSeeBit set when it is see-through.
template <class Cells>
__device__ __forceinline__ void observe(const Cells& cells, int ax, int ay, int dir, uint32_t carry,
                                        uint32_t (&w)[kObsWords]) {
  const int fx = dir_dx(dir), fy = dir_dy(dir);
  const int rx = -fy, ry = fx;
  uint32_t tri[kView * kView + 1];
  uint32_t seeds = 1u << 3;
#pragma unroll
  for (int j = kView - 1; j >= 0; --j) {
    const int bx = ax - 3 * rx + (6 - j) * fx, by = ay - 3 * ry + (6 - j) * fy;
    uint32_t see = 0;
#pragma unroll
    for (int i = 0; i < kView; ++i) {
      const uint32_t c = cells(bx + i * rx, by + i * ry);
      tri[j * kView + i] = c;
      see |= (c >> 31) << i;
    }
    uint32_t next;
    const uint32_t vis = visible_row(seeds, see, next);
#pragma unroll
    for (int i = 0; i < kView; ++i) {
      const int32_t keep = ((int32_t)(vis << (31 - i))) >> 31;
      tri[j * kView + i] &= (uint32_t)keep;
    }
    seeds = next;
  }
  tri[6 * kView + 3] = carry;   // the agent's own cell shows what it carries
  tri[kView * kView] = 0;
  // stream byte b belongs to cell b / 3; every dword spans two cells
#pragma unroll
  for (int d = 0; d < kObsWords; ++d) {
    const int k = (4 * d) / 3, off = (4 * d) % 3;
    const uint32_t sel = off == 0 ? 0x04020100u : (off == 1 ? 0x05040201u : 0x06050402u);
    w[d] = __builtin_amdgcn_perm(tri[k + 1], tri[k], sel);
  }
}

// Writes the lane's 147-byte record to stage[147 * lane ...] exactly: the
// record is realigned to the lane's byte offset with byte permutes; each
// dword shared by two neighbouring lanes is written by the higher lane,
// which takes the lower lane's tail through a cross-lane shuffle.
__device__ __forceinline__ void stage_record(uint8_t* stage, int lane, const uint32_t (&w)[kObsWords]) {
  const uint32_t s = (uint32_t)(kObsBytes * lane);
  const uint32_t m = s & 3u;
  uint32_t* base = reinterpret_cast<uint32_t*>(stage) + (s >> 2);
  const uint32_t sel = 0x07060504u - m * 0x01010101u;
  uint32_t u[kObsWords + 1];
  uint32_t prev = 0;
#pragma unroll
  for (int q = 0; q <= kObsWords; ++q) {
    const uint32_t cur = q < kObsWords ? w[q] : 0u;
    u[q] = __builtin_amdgcn_perm(cur, prev, sel);
    prev = cur;
  }
  const int last = (int)((m + kObsBytes - 1) >> 2);   // 36 or 37
  const uint32_t tail = last == kObsWords ? u[kObsWords] : u[kObsWords - 1];
  const uint32_t lower_tail = (uint32_t)__shfl_up((int)tail, 1, kWave);
  const bool last_owned = m == 1;                      // record ends on a dword boundary
  base[0] = m == 0 ? u[0] : (u[0] | lower_tail);
#pragma unroll
  for (int q = 1; q < kObsWords - 1; ++q) base[q] = u[q];
  if (last == kObsWords) {
    base[kObsWords - 1] = u[kObsWords - 1];
    if (last_owned) base[kObsWords] = u[kObsWords];
  } else if (last_owned) {
    base[kObsWords - 1] = u[kObsWords - 1];
  }
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Copies n_envs staged records (n_envs * 147 bytes) to dst.
__device__ __forceinline__ void copy_out(const uint8_t* stage, uint8_t* dst, int n_envs, int lane) {
  const int bytes = n_envs * kObsBytes;
  if (((reinterpret_cast<uintptr_t>(dst) & 15) == 0) && (bytes & 15) == 0) {
    const u32x4* src = reinterpret_cast<const u32x4*>(stage);
    u32x4* out = reinterpret_cast<u32x4*>(dst);
    for (int c = lane; c < (bytes >> 4); c += kWave) __builtin_nontemporal_store(src[c], out + c);
  } else {
    for (int b = lane; b < bytes; b += kWave) dst[b] = stage[b];
  }
}

// ---------------------------------------------------------------------------
// Plain kernel
// ---------------------------------------------------------------------------
struct HbmCells {
  const uint8_t* g;
  int S;
  __device__ __forceinline__ uint32_t operator()(int x, int y) const {
    if ((unsigned)x >= (unsigned)S || (unsigned)y >= (unsigned)S) return kCellWall;
    const uint8_t* p = g + 3 * (y * S + x);
    const uint32_t tri = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
    return tri | see_through(tri);
  }
};

__device__ __forceinline__ void store_triple(uint8_t* p, uint32_t tri) {
  p[0] = (uint8_t)tri;
  p[1] = (uint8_t)(tri >> 8);
  p[2] = (uint8_t)(tri >> 16);
}

struct PlainArgs {
  EnvTables env;
  StateBufs st;
  const uint8_t* actions;
  uint64_t call;
  int32_t reset_all;
  TrajBufs out;
  int32_t row;
};

__global__ __launch_bounds__(kWave) void k_plain(PlainArgs a) {
  __shared__ __align__(16) uint8_t stage[kStageBytes];
  const int lane = threadIdx.x;
  const int e0 = blockIdx.x * kWave;
  const int e = e0 + lane;
  const int N = a.env.n;
  const bool active = e < N;
  const int n_here = min(kWave, N - e0);

  uint32_t fam = 0;
  int S = 5, T = 1, x = 1, y = 1, dir = 0, t = 0;
  uint32_t carry = kCellEmpty, episode = 0, rid = 0;
  bool done_prev = false;
  uint2 seed = make_uint2(0, 0);
  uint8_t* g = a.st.grid;
  if (active) {
    const uint32_t meta = a.env.meta[e];
    fam = meta & 0xFF;
    S = (int)((meta >> 8) & 0xFF);
    T = a.env.max_steps[e];
    seed = a.env.seed[e];
    rid = a.env.rng_id[e];
    g = a.st.grid + a.env.grid_off[e];
    if (!a.reset_all) {
      x = a.st.x[e];
      y = a.st.y[e];
      dir = a.st.dir[e];
      t = a.st.t[e];
      carry = (uint32_t)a.st.carry[e];
      episode = a.st.episode[e];
      done_prev = a.st.done_prev[e] != 0;
    }
  }
  const bool do_reset = active && (a.reset_all || done_prev);
  Layout L{};
  if (do_reset) {
    episode = a.reset_all ? 0u : episode + 1u;
    L = make_layout(fam, S, seed, rid, episode);
    x = L.ax;
    y = L.ay;
    dir = L.dir;
    t = 0;
    carry = kCellEmpty;
  }
  // the wave writes every resetting env's new grid together, 32 cells a row
  uint64_t pending = __ballot(do_reset);
  while (pending) {
    const int r = __ffsll((unsigned long long)pending) - 1;
    pending &= pending - 1;
    const Layout Lr = bcast_layout(L, r);
    const uint64_t gr = ((uint64_t)(uint32_t)bcast((int)(uint32_t)reinterpret_cast<uint64_t>(g), r)) |
                        ((uint64_t)(uint32_t)bcast((int)(uint32_t)(reinterpret_cast<uint64_t>(g) >> 32), r) << 32);
    uint8_t* gp = reinterpret_cast<uint8_t*>(gr);
    const int xx = lane & 31;
    for (int yy = lane >> 5; yy < Lr.S; yy += 2)
      if (xx < Lr.S) store_triple(gp + 3 * (yy * Lr.S + xx), layout_cell(Lr, xx, yy));
  }
  __threadfence_block();
  __syncthreads();

  float reward = 0.0f;
  uint32_t flags = 0, act_rec = kActionNone;
  if (active && !do_reset) {
    uint32_t act;
    if (a.actions) {
      act = a.actions[e];
    } else {
      act = bounded(pick4(policy_block(seed, rid, a.call), (uint32_t)(a.call & 3)), 7u);
    }
    const int fx = x + dir_dx(dir), fy = y + dir_dy(dir);
    const HbmCells cells{g, S};
    const uint32_t front = cells(fx, fy);
    const ActResult r = intervene(act, x, y, dir, carry, front, fx, fy);
    if (r.front_changed) store_triple(g + 3 * (fy * S + fx), r.new_front);
    t += 1;
    const bool trunc = t >= T;
    reward = r.terminated ? goal_reward(t, T, a.env.reward_mode) : 0.0f;
    flags = (r.terminated ? kFlagTerminated : 0u) | (trunc ? kFlagTruncated : 0u);
    done_prev = r.terminated || trunc;
    act_rec = act & 0xFF;
  } else if (do_reset) {
    flags = kFlagFirst;
    done_prev = false;
  }

  const size_t rowN = (size_t)a.row * (size_t)N;
  if (a.out.obs) {
    uint32_t w[kObsWords];
    if (active) {
      observe(HbmCells{g, S}, x, y, dir, carry, w);
    } else {
#pragma unroll
      for (int q = 0; q < kObsWords; ++q) w[q] = 0;
    }
    stage_record(stage, lane, w);
    __syncthreads();
    copy_out(stage, a.out.obs + (rowN + (size_t)e0) * kObsBytes, n_here, lane);
  }
  if (active && a.out.reward) {
    a.out.reward[rowN + e] = reward;
    a.out.flags[rowN + e] = (uint8_t)flags;
    a.out.action[rowN + e] = (uint8_t)act_rec;
  }
  if (active) {
    a.st.x[e] = x;
    a.st.y[e] = y;
    a.st.dir[e] = dir;
    a.st.t[e] = t;
    a.st.carry[e] = (int32_t)carry;
    a.st.episode[e] = episode;
    a.st.done_prev[e] = done_prev ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// Fused kernel
// ---------------------------------------------------------------------------
// One byte per cell in LDS: bits 0-3 type (11 = locked door), bits 4-6
// colour, bit 7 closed door.  A 256-entry table maps codes back to triples
// (with the see-through bit).
__device__ __forceinline__ uint32_t code_of(uint32_t tri) {
  const uint32_t type = tri & 0xF, colour = (tri >> 8) & 7, state = (tri >> 16) & 0xFF;
  const bool door = type == kDoor;
  const uint32_t nib = (door && state == kLocked) ? 11u : type;
  return nib | (colour << 4) | ((door && state == kClosed) ? 0x80u : 0u);
}

__device__ __forceinline__ uint32_t triple_of_code(uint32_t code) {
  const uint32_t nib = code & 15, colour = (code >> 4) & 7;
  uint32_t tri;
  if (nib == 11) tri = kDoor | (colour << 8) | (kLocked << 16);
  else if (nib == kDoor) tri = kDoor | (colour << 8) | (((code >> 7) ? kClosed : kOpen) << 16);
  else tri = nib | (colour << 8);
  return tri | see_through(tri);
}

constexpr int kTableBytes = 256 * 4;
constexpr int kStageOff = kTableBytes;
constexpr int kGridOff = kStageOff + kStageBytes;  // 10432, 16-aligned
// A view reaches at most 6 cells ahead and 3 to the side of an interior
// agent, i.e. at most 5 rows and 5 columns outside an S <= 32 grid: with
// row-major indexing that is within 5 * 32 + 5 = 165 bytes before or after
// the grid.  Such cells are never visible (the wall border blocks sight),
// so only their addresses must stay inside the allocation.
constexpr int kMargin = 192;

struct LdsCells {
  const uint8_t* codes;   // this env's grid codes
  const uint32_t* table;
  int S;
  __device__ __forceinline__ uint32_t operator()(int x, int y) const {
    return table[codes[y * S + x]];
  }
};

struct FusedArgs {
  EnvTables env;
  TileTables tiles;
  StateBufs st;
  const uint8_t* actions;   // [k_steps][N] or nullptr
  uint64_t call0;
  int32_t k_steps;
  TrajBufs out;
  int32_t row0;
};

__device__ __forceinline__ int wave_excl_scan(int v, int lane, int& total) {
  int incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int n = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += n;
  }
  total = __shfl(incl, kWave - 1, kWave);
  return incl - v;
}

__global__ __launch_bounds__(kWave) void k_fused(FusedArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  uint32_t* table = reinterpret_cast<uint32_t*>(lds);
  uint8_t* stage = lds + kStageOff;
  uint8_t* codes = lds + kGridOff + kMargin;
  const int lane = threadIdx.x;
  const int N = a.env.n;

  for (int c = lane; c < 256; c += kWave) table[c] = triple_of_code((uint32_t)c);
  __syncthreads();

  for (int tile = blockIdx.x; tile < a.tiles.n_tiles; tile += gridDim.x) {
    const int e0 = tile * kWave;
    const int e = e0 + lane;
    const bool active = e < N;
    const int n_here = min(kWave, N - e0);

    uint32_t fam = 0;
    int S = 0, T = 1, x = 1, y = 1, dir = 0, t = 0;
    uint32_t carry = kCellEmpty, episode = 0, rid = 0;
    bool done_prev = false;
    uint2 seed = make_uint2(0, 0);
    uint64_t goff = 0;
    if (active) {
      const uint32_t meta = a.env.meta[e];
      fam = meta & 0xFF;
      S = (int)((meta >> 8) & 0xFF);
      T = a.env.max_steps[e];
      seed = a.env.seed[e];
      rid = a.env.rng_id[e];
      goff = a.env.grid_off[e];
      x = a.st.x[e];
      y = a.st.y[e];
      dir = a.st.dir[e];
      t = a.st.t[e];
      carry = (uint32_t)a.st.carry[e];
      episode = a.st.episode[e];
      done_prev = a.st.done_prev[e] != 0;
    }
    int tile_cells;
    const int my_off = wave_excl_scan(S * S, lane, tile_cells);
    uint8_t* my_codes = codes + my_off;
    // the tile's grids are contiguous in HBM: stage them as codes
    {
      const uint64_t g0 = (uint64_t)__shfl((long long)goff, 0, kWave);
      const uint8_t* src = a.st.grid + g0;
      for (int c = lane; c < tile_cells; c += kWave) {
        const uint32_t tri = (uint32_t)src[3 * c] | ((uint32_t)src[3 * c + 1] << 8) |
                             ((uint32_t)src[3 * c + 2] << 16);
        codes[c] = (uint8_t)code_of(tri);
      }
    }
    __syncthreads();

    uint4 pol = make_uint4(0, 0, 0, 0);
    for (int s = 0; s < a.k_steps; ++s) {
      const uint64_t call = a.call0 + (uint64_t)s;
      if (!a.actions && (s == 0 || (call & 3) == 0)) pol = policy_block(seed, rid, call);

      const bool do_reset = active && done_prev;
      Layout L{};
      if (do_reset) {
        episode += 1u;
        L = make_layout(fam, S, seed, rid, episode);
        x = L.ax;
        y = L.ay;
        dir = L.dir;
        t = 0;
        carry = kCellEmpty;
      }
      uint64_t pending = __ballot(do_reset);
      if (pending) {
        while (pending) {
          const int r = __ffsll((unsigned long long)pending) - 1;
          pending &= pending - 1;
          const Layout Lr = bcast_layout(L, r);
          uint8_t* gp = codes + bcast(my_off, r);
          const int xx = lane & 31;
          for (int yy = lane >> 5; yy < Lr.S; yy += 2)
            if (xx < Lr.S) gp[yy * Lr.S + xx] = (uint8_t)code_of(layout_cell(Lr, xx, yy));
        }
        __syncthreads();
      }

      float reward = 0.0f;
      uint32_t flags = 0, act_rec = kActionNone;
      if (active && !do_reset) {
        const uint32_t act = a.actions ? (uint32_t)a.actions[(size_t)s * N + e]
                                       : bounded(pick4(pol, (uint32_t)(call & 3)), 7u);
        const int fx = x + dir_dx(dir), fy = y + dir_dy(dir);
        const uint32_t front = table[my_codes[fy * S + fx]];
        const ActResult r = intervene(act, x, y, dir, carry, front, fx, fy);
        if (r.front_changed) my_codes[fy * S + fx] = (uint8_t)code_of(r.new_front);
        t += 1;
        const bool trunc = t >= T;
        reward = r.terminated ? goal_reward(t, T, a.env.reward_mode) : 0.0f;
        flags = (r.terminated ? kFlagTerminated : 0u) | (trunc ? kFlagTruncated : 0u);
        done_prev = r.terminated || trunc;
        act_rec = act & 0xFF;
      } else if (do_reset) {
        flags = kFlagFirst;
        done_prev = false;
      }

      const int row = (a.row0 + s) % a.out.rows;
      const size_t rowN = (size_t)row * (size_t)N;
      if (a.out.obs) {
        uint32_t w[kObsWords];
        if (active) {
          observe(LdsCells{my_codes, table, S}, x, y, dir, carry, w);
        } else {
#pragma unroll
          for (int q = 0; q < kObsWords; ++q) w[q] = 0;
        }
        stage_record(stage, lane, w);
        __syncthreads();
        copy_out(stage, a.out.obs + (rowN + (size_t)e0) * kObsBytes, n_here, lane);
      }
      if (active) {
        a.out.reward[rowN + e] = reward;
        a.out.flags[rowN + e] = (uint8_t)flags;
        a.out.action[rowN + e] = (uint8_t)act_rec;
      }
      __syncthreads();
    }

    // write the chunk's final state back
    {
      const uint64_t g0 = (uint64_t)__shfl((long long)goff, 0, kWave);
      uint8_t* dst = a.st.grid + g0;
      for (int c = lane; c < tile_cells; c += kWave) {
        const uint32_t tri = table[codes[c]];
        dst[3 * c] = (uint8_t)tri;
        dst[3 * c + 1] = (uint8_t)(tri >> 8);
        dst[3 * c + 2] = (uint8_t)(tri >> 16);
      }
    }
    if (active) {
      a.st.x[e] = x;
      a.st.y[e] = y;
      a.st.dir[e] = dir;
      a.st.t[e] = t;
      a.st.carry[e] = (int32_t)carry;
      a.st.episode[e] = episode;
      a.st.done_prev[e] = done_prev ? 1 : 0;
    }
    __syncthreads();
  }
}

}  // namespace

size_t fused_lds_bytes(int32_t max_tile_cells) {
  size_t b = (size_t)kGridOff + 2 * kMargin + (size_t)max_tile_cells;
  return (b + 15) & ~(size_t)15;
}

hipError_t launch_plain(const EnvTables& env, const StateBufs& st, const uint8_t* actions,
                        uint64_t call, int reset_all, const TrajBufs& out, int32_t row,
                        hipStream_t stream) {
  PlainArgs a{env, st, actions, call, reset_all, out, row};
  const int blocks = (env.n + kWave - 1) / kWave;
  hipLaunchKernelGGL(k_plain, dim3(blocks), dim3(kWave), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_fused(const EnvTables& env, const TileTables& tiles, const StateBufs& st,
                        const uint8_t* actions, uint64_t call0, int32_t k_steps,
                        const TrajBufs& out, int32_t row0, int32_t grid_blocks,
                        hipStream_t stream) {
  FusedArgs a{env, tiles, st, actions, call0, k_steps, out, row0};
  const size_t lds = fused_lds_bytes(tiles.max_tile_cells);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_fused, dim3(grid_blocks), dim3(kWave), lds, stream, a);
  return hipGetLastError();
}

}  // namespace gx
