// kernels.hip -- gfx950 kernels of the batched gridworld environment step.
//
// The step is NAVIX's interaction protocol (arXiv 2407.19396, Sec. 3.2.2:
// step(timestep, action) with autoreset; reset pads action -1, reward 0)
// applied to MiniGrid's dynamics, which the paper reproduces exactly
// (Sec. 3.2.1): the intervention / transition / observation / reward /
// termination systems of Table "systems" and App. A over the entities of
// Table "entities", for every family of Table "envs".
//
// Two kernels share the device functions below:
//   k_plain  -- one launch per step; one env per lane; state, grid and
//               outputs in HBM; view cells read straight from the grid.
//   k_fused  -- persistent; each workgroup takes tiles of 64 envs of any
//               mix of sizes, stages their grids in LDS as one byte per
//               cell, runs K steps with the pose in registers, writes one
//               trajectory record per env-step, then writes the state back.
//               Its serving variant also admits and resets new requests.
// Both stage the first-person observations of a wave through LDS so that
// the wave's records leave as one contiguous, 16-byte-vectorised block;
// whole-grid observations leave the same way, packed like the grids.
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
constexpr int kHalfStageBytes = kStageBytes / 2;    // 4704, a multiple of 16
// the fused kernel's record stage: 32 records behind up to 48 bytes carried
// over from the previous piece (see k_fused)
constexpr int kRecStageBytes = kHalfStageBytes + 48;
constexpr int kObsWords = 37;                       // ceil(147 / 4)
constexpr int kCatBytes = kView * kView;            // categorical record: 49
constexpr int kCatWords = 13;                       // ceil(49 / 4)

// Cell triples are packed as type | colour << 8 | state << 16 (MiniGrid's
// object, colour and state indices).  Bit 31 marks a see-through cell.
constexpr uint32_t kEmpty = 1, kWall = 2, kDoor = 4, kKey = 5, kBall = 6, kBox = 7, kGoal = 8,
                   kLava = 9;
constexpr uint32_t kGreen = 1, kGrey = 5;
constexpr uint32_t kOpen = 0, kClosed = 1, kLocked = 2;
constexpr uint32_t kSeeBit = 1u << 31;
constexpr uint32_t kSeeBits = 0xFE000000u;   // see flags of view columns 0-6 at bits 31-25
constexpr uint32_t kCellWall = kWall | (kGrey << 8);
constexpr uint32_t kCellEmpty = kEmpty;
constexpr uint32_t kCellGoal = kGoal | (kGreen << 8);

constexpr uint32_t kFlagTerminated = 1, kFlagTruncated = 2, kFlagFirst = 4;
constexpr uint32_t kActionNone = 0xFF;

enum : uint32_t { kLeft = 0, kRight = 1, kForward = 2, kPickup = 3, kDrop = 4, kToggle = 5 };
enum : uint32_t {
  kFamEmpty = 0, kFamTwoRoom = 1, kFamFourRooms = 2,
  kFamLavaGap = 3, kFamCrossings = 4, kFamDistShift = 5, kFamDynObs = 6, kFamGoToDoor = 7,
  kFamKeyCorridor = 8
};
constexpr int kMaxObst = 8;
constexpr uint32_t kBlue = 2;
constexpr uint32_t kCellBall = kBall | (kBlue << 8);

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

// Random-policy words of an env's call block `call >> 2`: counter (id,
// block, 0, 1); call = the env's step calls since its reset.
__device__ __forceinline__ uint4 policy_block(uint2 seed, uint32_t rng_id, uint32_t call) {
  return philox10(make_uint4(rng_id, call >> 2, 0u, 1u), seed);
}

// ---------------------------------------------------------------------------
// Start states (reset(key) of Sec. 3.2.2; the families of Table "envs").
// Layout parameters come from the layout stream, counter (id, episode,
// block, 0), in draw order; "uniform placement" picks the k-th free cell
// in row-major order, which every family below reaches in closed form.
// ---------------------------------------------------------------------------
struct Layout {
  int fam, S;
  int a, b, c, d;      // TwoRoom: a = wall column, b = door row; FourRooms: the 4 openings;
                       // LavaGap: a = lava column, b = gap row; DistShift: a = second lava row;
                       // GoToDoor: the doors' positions along the top, right, bottom, left walls
  int colour;          // TwoRoom, KeyCorridor: locked door / key colour; GoToDoor: door i's
                       // colour at bits 4i..4i+3
  int kx, ky;          // TwoRoom, KeyCorridor: key; GoToDoor: the room's width and height
  int gx, gy;          // goal
  int ax, ay, dir;     // agent
  uint32_t vmask, hmask;   // Crossings: river columns / rows (bit = coordinate)
  uint64_t vopen, hopen;   // Crossings: opening row of each river column, opening column
                           // of each river row, 5 bits each in ascending river order
  uint32_t ob[4];          // Dynamic-Obstacles: ball b at bytes 2b (x), 2b + 1 (y); 0xFF unused
  uint32_t kd[3];          // KeyCorridor: the doors between rooms, one byte each (see below)
};

// (x, y) of ball b from a packed obstacle list
__device__ __forceinline__ uint32_t obst_at(const uint32_t (&ob)[4], int b) {
  return (ob[b >> 1] >> (16 * (b & 1))) & 0xFFFFu;
}

__device__ __forceinline__ void obst_set(uint32_t (&ob)[4], int b, uint32_t x, uint32_t y) {
  const int sh = 16 * (b & 1);
  ob[b >> 1] = (ob[b >> 1] & ~(0xFFFFu << sh)) | ((x | (y << 8)) << sh);
}

__device__ __forceinline__ bool is_ball(const Layout& L, int x, int y) {
  const uint32_t xy = (uint32_t)x | ((uint32_t)y << 8);
  bool hit = false;
#pragma unroll
  for (int b = 0; b < kMaxObst; ++b) hit = hit || obst_at(L.ob, b) == xy;
  return hit;
}

// Layout-stream draws taken in order, one Philox block per 4 words.
struct DrawStream {
  uint2 seed;
  uint32_t id, episode, w;
  uint4 block;
  __device__ __forceinline__ uint32_t next(uint32_t n) {
    if ((w & 3u) == 0) block = philox10(make_uint4(id, episode, w >> 2, 0u), seed);
    const uint32_t r = bounded(pick4(block, w & 3u), n);
    ++w;
    return r;
  }
};

// position of the k-th (0-based) set bit of m
__device__ __forceinline__ int kth_bit(uint32_t m, int k) {
  for (int i = 0; i < k; ++i) m &= m - 1u;
  return __builtin_ctz(m);
}

// Crossings(S, N): N of the M = S - 3 candidate rivers (columns 2, 4, ..,
// S - 3, then rows 2, 4, .., S - 3) by a partial Fisher-Yates shuffle, then
// a monotone path of room moves, each opening one cell of the river it
// crosses (Table "envs", Crossings; lava of Table "entities").  The shuffle
// keeps only the positions it touched: entry k records that position
// mkey[k] now holds candidate mval[k].
constexpr int kMaxRivers = 8;

struct Rivers {
  uint32_t vmask, hmask;
  uint64_t vopen, hopen;
};

__device__ __noinline__ Rivers crossings_layout(int S, int N, uint2 seed, uint32_t rng_id,
                                                uint32_t episode) {
  DrawStream ds{seed, rng_id, episode, 0u, make_uint4(0, 0, 0, 0)};
  const int M = S - 3, h = M / 2;
  int mkey[kMaxRivers], mval[kMaxRivers];
  Rivers R{0u, 0u, 0ull, 0ull};
#pragma unroll
  for (int k = 0; k < kMaxRivers; ++k) {
    if (k < N) {
      const int r = k + (int)ds.next((uint32_t)(M - k));
      int vk = k, vr = r;
#pragma unroll
      for (int j = 0; j < k; ++j) {
        vk = mkey[j] == k ? mval[j] : vk;
        vr = mkey[j] == r ? mval[j] : vr;
      }
      mkey[k] = r;
      mval[k] = vk;
      if (vr < h) R.vmask |= 1u << (2 + 2 * vr);
      else R.hmask |= 1u << (2 + 2 * (vr - h));
    }
  }
  const int nv = __builtin_popcount(R.vmask), nh = __builtin_popcount(R.hmask);
  int ci = 0, rj = 0;
  for (int q = 0; q < N; ++q) {
    const int rv = nv - ci, rh = nh - rj;
    if ((int)ds.next((uint32_t)(rv + rh)) < rv) {
      const int lo = rj == 0 ? 0 : kth_bit(R.hmask, rj - 1);
      const int hi = rj == nh ? S - 1 : kth_bit(R.hmask, rj);
      const uint64_t y = (uint64_t)(lo + 1 + (int)ds.next((uint32_t)(hi - lo - 1)));
      R.vopen |= y << (5 * ci);
      ++ci;
    } else {
      const int lo = ci == 0 ? 0 : kth_bit(R.vmask, ci - 1);
      const int hi = ci == nv ? S - 1 : kth_bit(R.vmask, ci);
      const uint64_t x = (uint64_t)(lo + 1 + (int)ds.next((uint32_t)(hi - lo - 1)));
      R.hopen |= x << (5 * rj);
      ++rj;
    }
  }
  return R;
}

// whether interior cell (x, y) of a Crossings layout is lava
__device__ __forceinline__ bool crossings_lava(const Layout& L, int x, int y) {
  bool lava = false;
  if ((L.vmask >> x) & 1u) {
    const int rank = __builtin_popcount(L.vmask & ((1u << x) - 1u));
    lava = y != (int)((L.vopen >> (5 * rank)) & 31u);
  }
  if ((L.hmask >> y) & 1u) {
    const int rank = __builtin_popcount(L.hmask & ((1u << y) - 1u));
    lava = lava || x != (int)((L.hopen >> (5 * rank)) & 31u);
  }
  return lava;
}

// q = k / w, r = k % w for k < 2^16 and 1 <= w <= 32.  The single-precision
// quotient is within a few ulp of k / w, far less than the 1 / w distance
// between its fractional part and the next integer when k % w != 0; when
// k % w == 0 it may fall just short of q, which the correction repairs.
__device__ __forceinline__ void small_divmod(uint32_t k, uint32_t w, uint32_t& q, uint32_t& r) {
  q = (uint32_t)((float)k * __builtin_amdgcn_rcpf((float)w));
  r = k - q * w;
  const bool under = r >= w;
  q += under ? 1u : 0u;
  r -= under ? w : 0u;
}

// KeyCorridor(S = 3s - 2, R rows of rooms): walls between two rooms, one
// byte each in L.kd (byte e of word e / 4): bit 7 set when the wall has a
// door, bits 4-6 its colour, bits 0-3 its position along the wall.  Walls
// between columns i and i + 1 in row j: e = 2j + i; walls between rows jw
// and jw + 1 in column 0 or 2: e = 6 + 2 jw + i / 2 (column 1 is the open
// hallway).  The locked door is the wall e = 2 rl + 1 of the locked row rl.
__device__ __forceinline__ uint32_t kc_byte(const uint32_t (&kd)[3], int e) {
  const uint64_t lo = (uint64_t)kd[0] | ((uint64_t)kd[1] << 32);
  return e < 8 ? (uint32_t)(lo >> (8 * e)) & 0xFFu : (kd[2] >> (8 * (e - 8))) & 0xFFu;
}

// rooms reachable from room `from` (bit j * 3 + i) through the open walls:
// right[r] / down[r] bits say room r connects to r + 1 / r + 3
__device__ __forceinline__ uint32_t kc_reach(uint32_t from, uint32_t right, uint32_t down) {
  uint32_t r = from;
#pragma unroll
  for (int it = 0; it < 8; ++it)
    r |= ((r & right) << 1) | ((r >> 1) & right) | ((r & down) << 3) | ((r >> 3) & down);
  return r;
}

struct KcLayout {
  int rl, colour, gx, gy, kx, ky, ax, ay, dir;
  uint32_t kd[3];
};

__device__ __noinline__ KcLayout keycorridor_layout(int S, int R, uint2 seed, uint32_t rng_id,
                                                    uint32_t episode) {
  DrawStream ds{seed, rng_id, episode, 0u, make_uint4(0, 0, 0, 0)};
  const int st = (S - 1) / 3, inner = st - 1;
  // door positions of walls e = 0..9 (the table's numbering), 4 bits each
  uint64_t pos = 0;
  for (int j = 0; j < R; ++j)
    for (int i = 0; i < 3; ++i) {
      if (i < 2) pos |= (uint64_t)ds.next((uint32_t)inner) << (4 * (2 * j + i));
      if (j < R - 1) {
        const uint64_t p = ds.next((uint32_t)inner);   // the hallway's wall draws one too
        if (i != 1) pos |= p << (4 * (6 + 2 * j + (i >> 1)));
      }
    }
  KcLayout K;
  K.rl = (int)ds.next((uint32_t)R);
  K.colour = (int)ds.next(6u);
  // the door table: bytes 0-7 in lo, 8-9 in hi
  uint64_t lo = 0;
  uint32_t hi = 0;
  const int el = 2 * K.rl + 1;   // < 8
  lo |= (uint64_t)(0x80u | ((uint32_t)K.colour << 4) | (uint32_t)((pos >> (4 * el)) & 15u)) << (8 * el);
  uint32_t q, r;
  small_divmod(ds.next((uint32_t)(inner * inner)), (uint32_t)inner, q, r);
  K.gx = 2 * st + 1 + (int)r;
  K.gy = K.rl * st + 1 + (int)q;
  const int rk = (int)ds.next((uint32_t)R);
  small_divmod(ds.next((uint32_t)(inner * inner)), (uint32_t)inner, q, r);
  K.kx = 1 + (int)r;
  K.ky = rk * st + 1 + (int)q;
  const int ra = R / 2;
  small_divmod(ds.next((uint32_t)(inner * inner)), (uint32_t)inner, q, r);
  K.ax = st + 1 + (int)r;
  K.ay = ra * st + 1 + (int)q;
  K.dir = (int)ds.next(4u);
  // connect every room (MiniGrid's connect_all), the locked room excepted
  const uint32_t all = (1u << (3 * R)) - 1u;
  uint32_t right = 1u << (3 * K.rl + 1), down = 0u;   // the locked door
  for (int j = 0; j + 1 < R; ++j) down |= 1u << (3 * j + 1);   // the hallway
  for (int it = 0; it < 1024; ++it) {
    if (kc_reach(1u << (3 * ra + 1), right, down) == all) break;
    const int i = (int)ds.next(3u), j = (int)ds.next((uint32_t)R), k = (int)ds.next(4u);
    const int i2 = i + (k == 0) - (k == 2), j2 = j + (k == 1) - (k == 3);
    if (i2 < 0 || i2 > 2 || j2 < 0 || j2 >= R) continue;
    const bool horiz = j2 == j;
    const int room = horiz ? 3 * j + min(i, i2) : 3 * min(j, j2) + i;
    if (((horiz ? right : down) >> room) & 1u) continue;
    if ((i == 2 && j == K.rl) || (i2 == 2 && j2 == K.rl)) continue;
    const uint32_t c = ds.next(6u);
    const int e = horiz ? 2 * j + min(i, i2) : 6 + 2 * min(j, j2) + (i >> 1);
    if (horiz) right |= 1u << room;
    else down |= 1u << room;
    const uint32_t v = 0x80u | (c << 4) | (uint32_t)((pos >> (4 * e)) & 15u);
    if (e < 8) lo |= (uint64_t)v << (8 * e);
    else hi |= v << (8 * (e - 8));
  }
  K.kd[0] = (uint32_t)lo;
  K.kd[1] = (uint32_t)(lo >> 32);
  K.kd[2] = hi;
  return K;
}

// idx-th free cell, row-major, of a four-room grid of side S = 2m + 1 with
// openings (m, g1), (m, g2) in the vertical wall (g1 < m < g2) and
// (g3, m), (g4, m) in the horizontal one.  Rows other than m hold S - 3 free
// cells (the wall column removed), S - 2 in the opening rows g1 and g2; row
// m holds the two openings.
__device__ __forceinline__ void fourrooms_cell(int S, int m, int g1, int g2, int g3, int g4,
                                               uint32_t idx, int& x, int& y) {
  const uint32_t W = (uint32_t)(S - 3);
  const uint32_t top = (uint32_t)(m - 1) * W + 1u;   // free cells in rows 1 .. m-1
  if (idx - top < 2u) {                              // row m
    y = m;
    x = idx == top ? g3 : g4;
    return;
  }
  const bool low = idx >= top;
  const int row0 = low ? m + 1 : 1, gap = low ? g2 : g1;
  const uint32_t k = low ? idx - top - 2u : idx;
  const uint32_t before = (uint32_t)(gap - row0) * W;   // cells in the rows above the gap row
  if (k - before <= W) {                                // the gap row: every interior cell
    y = gap;
    x = 1 + (int)(k - before);
    return;
  }
  uint32_t q, r;
  small_divmod(k < before ? k : k - 1u, W, q, r);
  y = row0 + (int)q;
  x = 1 + (int)r;
  x += x >= m ? 1 : 0;
}

// meta = family | side << 8 | parameter << 16 (Crossings: rivers; DistShift:
// variant; Dynamic-Obstacles: balls; KeyCorridor: rows of rooms).  The lava
// families and Dynamic-Obstacles start at (1, 1) facing east.
__device__ Layout make_layout(uint32_t meta, uint2 seed, uint32_t rng_id, uint32_t episode) {
  const uint32_t fam = meta & 0xFF;
  const int S = (int)((meta >> 8) & 0xFF), param = (int)((meta >> 16) & 0xFF);
  Layout L;
  L.fam = (int)fam;
  L.S = S;
  L.a = L.b = L.c = L.d = -1;
  L.colour = 0;
  L.kx = L.ky = -1;
  L.gx = S - 2;
  L.gy = S - 2;
  L.vmask = L.hmask = 0;
  L.vopen = L.hopen = 0;
  L.ob[0] = L.ob[1] = L.ob[2] = L.ob[3] = 0xFFFFFFFFu;
  L.kd[0] = L.kd[1] = L.kd[2] = 0u;
  if (fam == kFamKeyCorridor) {
    const KcLayout K = keycorridor_layout(S, param, seed, rng_id, episode);
    L.a = K.rl;
    L.b = param;   // rows of rooms
    L.colour = K.colour;
    L.gx = K.gx;
    L.gy = K.gy;
    L.kx = K.kx;
    L.ky = K.ky;
    L.ax = K.ax;
    L.ay = K.ay;
    L.dir = K.dir;
    L.kd[0] = K.kd[0];
    L.kd[1] = K.kd[1];
    L.kd[2] = K.kd[2];
    return L;
  }
  if (fam == kFamDynObs) {
    // balls in order, ball b at the draw-b-th free interior cell other than
    // the agent's (1, 1): linear interior index c with c - #{earlier balls
    // <= c} = draw + 1, found by iterating c = draw + 1 + #{balls <= c}
    L.ax = L.ay = 1;
    L.dir = 0;
    const uint32_t w = (uint32_t)(S - 2);
    const uint4 w0 = philox10(make_uint4(rng_id, episode, 0u, 0u), seed);
    const uint4 w1 = param > 4 ? philox10(make_uint4(rng_id, episode, 1u, 0u), seed)
                               : make_uint4(0, 0, 0, 0);
    uint32_t p[kMaxObst];
#pragma unroll
    for (int b = 0; b < kMaxObst; ++b) {
      p[b] = 0xFFFFu;
      if (b < param) {
        const uint32_t word = pick4(b < 4 ? w0 : w1, (uint32_t)(b & 3));
        const uint32_t k = bounded(word, w * w - 2u - (uint32_t)b);
        uint32_t c = k + 1u;
#pragma unroll
        for (int it = 0; it < b; ++it) {
          uint32_t below = 0;
#pragma unroll
          for (int j = 0; j < b; ++j) below += p[j] <= c ? 1u : 0u;
          c = k + 1u + below;
        }
        p[b] = c;
        uint32_t q, r;
        small_divmod(c, w, q, r);
        obst_set(L.ob, b, 1u + r, 1u + q);
      }
    }
    return L;
  }
  if (fam == kFamGoToDoor) {
    // room w x h in the top-left corner, one closed door per wall (top x,
    // right y, bottom x, left y), four distinct colours by a partial
    // Fisher-Yates shuffle of the six, the mission the colour of door u(4),
    // the agent uniform over the room's interior; 13 words in draw order
    const uint4 w0 = philox10(make_uint4(rng_id, episode, 0u, 0u), seed);
    const uint4 w1 = philox10(make_uint4(rng_id, episode, 1u, 0u), seed);
    const uint4 w2 = philox10(make_uint4(rng_id, episode, 2u, 0u), seed);
    const uint4 w3 = philox10(make_uint4(rng_id, episode, 3u, 0u), seed);
    const int rw = 5 + (int)bounded(w0.x, (uint32_t)(S - 4));
    const int rh = 5 + (int)bounded(w0.y, (uint32_t)(S - 4));
    L.kx = rw;
    L.ky = rh;
    L.gx = L.gy = -1;   // no goal square
    L.a = 1 + (int)bounded(w0.z, (uint32_t)(rw - 2));
    L.b = 1 + (int)bounded(w0.w, (uint32_t)(rh - 2));
    L.c = 1 + (int)bounded(w1.x, (uint32_t)(rw - 2));
    L.d = 1 + (int)bounded(w1.y, (uint32_t)(rh - 2));
    uint32_t col = 0x543210u;   // colour k at bits 4k..4k+3
    const uint32_t sw[4] = {w1.z, w1.w, w2.x, w2.y};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t r = (uint32_t)k + bounded(sw[k], (uint32_t)(6 - k));
      const uint32_t ck = (col >> (4 * k)) & 15u, cr = (col >> (4 * r)) & 15u;
      col = (col & ~((15u << (4 * k)) | (15u << (4 * r)))) | (cr << (4 * k)) | (ck << (4 * r));
    }
    L.colour = (int)(col & 0xFFFFu);
    const uint32_t target = bounded(w2.z, 4u);
    L.ob[0] = 0xFFFFFF00u | ((col >> (4 * target)) & 15u);
    uint32_t q, r;
    small_divmod(bounded(w2.w, (uint32_t)((rw - 2) * (rh - 2))), (uint32_t)(rw - 2), q, r);
    L.ax = 1 + (int)r;
    L.ay = 1 + (int)q;
    L.dir = (int)bounded(w3.x, 4u);
    return L;
  }
  if (fam >= kFamLavaGap) {
    L.ax = L.ay = 1;
    L.dir = 0;
    if (fam == kFamLavaGap) {
      const uint4 w0 = philox10(make_uint4(rng_id, episode, 0u, 0u), seed);
      L.a = 2 + (int)bounded(w0.x, (uint32_t)(S - 4));
      L.b = 1 + (int)bounded(w0.y, (uint32_t)(S - 2));
    } else if (fam == kFamCrossings) {
      const Rivers R = crossings_layout(S, param, seed, rng_id, episode);
      L.vmask = R.vmask;
      L.hmask = R.hmask;
      L.vopen = R.vopen;
      L.hopen = R.hopen;
    } else {
      L.gy = 1;
      L.a = param == 1 ? 2 : S - 2;
    }
    return L;
  }
  const uint4 w0 = philox10(make_uint4(rng_id, episode, 0u, 0u), seed);
  const uint4 w1 = philox10(make_uint4(rng_id, episode, 1u, 0u), seed);
  if (fam == kFamEmpty) {
    const int w = S - 2;
    const uint32_t k = bounded(w0.x, (uint32_t)(w * w - 1));   // interior minus the last (goal) cell
    uint32_t q, r;
    small_divmod(k, (uint32_t)w, q, r);
    L.ax = 1 + (int)r;
    L.ay = 1 + (int)q;
    L.dir = (int)bounded(w0.y, 4u);
  } else if (fam == kFamTwoRoom) {
    L.a = 2 + (int)bounded(w0.x, (uint32_t)(S - 4));
    L.b = 1 + (int)bounded(w0.y, (uint32_t)(S - 3));
    L.colour = (int)bounded(w0.z, 6u);
    const uint32_t lw = (uint32_t)(L.a - 1), n = lw * (uint32_t)(S - 2);
    const uint32_t kk = bounded(w0.w, n);
    uint32_t q, r;
    small_divmod(kk, lw, q, r);
    L.kx = 1 + (int)r;
    L.ky = 1 + (int)q;
    uint32_t ka = bounded(w1.x, n - 1u);
    ka += ka >= kk ? 1u : 0u;
    small_divmod(ka, lw, q, r);
    L.ax = 1 + (int)r;
    L.ay = 1 + (int)q;
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
// GoToDoor door i's colour, or -1 when (x, y) holds no door
__device__ __forceinline__ int gotodoor_door(const Layout& L, int x, int y) {
  int i = -1;
  i = (y == 0 && x == L.a) ? 0 : i;
  i = (x == L.kx - 1 && y == L.b) ? 1 : i;
  i = (y == L.ky - 1 && x == L.c) ? 2 : i;
  i = (x == 0 && y == L.d) ? 3 : i;
  return i < 0 ? -1 : (int)(((uint32_t)L.colour >> (4 * i)) & 15u);
}

// content of KeyCorridor cell (x, y): rooms of stride st = (S - 1) / 3 in
// the top R * st + 1 rows, wall below; doors from the wall table
__device__ __forceinline__ uint32_t keycorridor_cell(const Layout& L, int x, int y) {
  const int st = (L.S - 1) / 3, R = L.b;
  if (y > R * st) return kCellWall;
  uint32_t qx, mx, qy, my;
  small_divmod((uint32_t)x, (uint32_t)st, qx, mx);
  small_divmod((uint32_t)y, (uint32_t)st, qy, my);
  if (mx != 0 && my != 0) {
    if (x == L.gx && y == L.gy) return kCellGoal;
    if (x == L.kx && y == L.ky) return kKey | ((uint32_t)L.colour << 8);
    return kCellEmpty;
  }
  if (mx == 0 && my == 0) return kCellWall;
  int e;
  uint32_t p;
  if (mx == 0) {   // a wall between columns qx - 1 and qx, in row qy
    if (qx == 0 || qx == 3) return kCellWall;
    e = 2 * (int)qy + (int)qx - 1;
    p = my - 1;
  } else {         // a wall between rows qy - 1 and qy, in column qx
    if (qy == 0 || (int)qy == R) return kCellWall;
    if (qx == 1) return kCellEmpty;   // the hallway
    e = 6 + 2 * ((int)qy - 1) + (int)(qx >> 1);
    p = mx - 1;
  }
  const uint32_t d = kc_byte(L.kd, e);
  if (!(d & 0x80u) || (d & 15u) != p) return kCellWall;
  const uint32_t state = e == 2 * L.a + 1 ? kLocked : kClosed;
  return kDoor | (((d >> 4) & 7u) << 8) | (state << 16);
}

__device__ __forceinline__ uint32_t layout_cell(const Layout& L, int x, int y) {
  const int S = L.S;
  if (L.fam == kFamKeyCorridor) return keycorridor_cell(L, x, y);
  if (L.fam == kFamGoToDoor) {
    const int dc = gotodoor_door(L, x, y);
    if (dc >= 0) return kDoor | ((uint32_t)dc << 8) | (kClosed << 16);
    return (x == 0 || y == 0 || x >= L.kx - 1 || y >= L.ky - 1) ? kCellWall : kCellEmpty;
  }
  if (x == 0 || y == 0 || x == S - 1 || y == S - 1) return kCellWall;
  if (x == L.gx && y == L.gy) return kCellGoal;
  if (L.fam == kFamTwoRoom) {
    if (x == L.a) return y == L.b ? (kDoor | ((uint32_t)L.colour << 8) | (kLocked << 16)) : kCellWall;
    if (x == L.kx && y == L.ky) return kKey | ((uint32_t)L.colour << 8);
  } else if (L.fam == kFamFourRooms) {
    const int m = S / 2;
    if (x == m) return (y == L.a || y == L.b) ? kCellEmpty : kCellWall;
    if (y == m) return (x == L.c || x == L.d) ? kCellEmpty : kCellWall;
  } else if (L.fam == kFamLavaGap) {
    if (x == L.a && y != L.b) return kLava;
  } else if (L.fam == kFamCrossings) {
    if (crossings_lava(L, x, y)) return kLava;
  } else if (L.fam == kFamDistShift) {
    if ((y == 1 || y == L.a) && x >= 3 && x <= S - 3) return kLava;
  } else if (L.fam == kFamDynObs) {
    if (is_ball(L, x, y)) return kCellBall;
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
  o.vmask = (uint32_t)bcast((int)L.vmask, r);
  o.hmask = (uint32_t)bcast((int)L.hmask, r);
  o.vopen = (uint64_t)(uint32_t)bcast((int)(uint32_t)L.vopen, r) |
            ((uint64_t)(uint32_t)bcast((int)(L.vopen >> 32), r) << 32);
  o.hopen = (uint64_t)(uint32_t)bcast((int)(uint32_t)L.hopen, r) |
            ((uint64_t)(uint32_t)bcast((int)(L.hopen >> 32), r) << 32);
#pragma unroll
  for (int i = 0; i < 4; ++i) o.ob[i] = (uint32_t)bcast((int)L.ob[i], r);
#pragma unroll
  for (int i = 0; i < 3; ++i) o.kd[i] = (uint32_t)bcast((int)L.kd[i], r);
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
  bool goal;      // the task achieved: the goal reached, or (GoToDoor) done at the mission's door
  bool penalty;   // ended with reward -1: walked into lava, or (Dynamic-Obstacles)
                  // stepped forward at a ball or wall
};

__device__ __forceinline__ ActResult intervene(uint32_t act, int& x, int& y, int& dir, uint32_t& carry,
                                               uint32_t front, int fx, int fy) {
  // every lane of a wave holds its own action, so the rules are evaluated
  // as selects rather than branches
  const uint32_t type = front & 0xFF, colour = (front >> 8) & 0xFF, state = (front >> 16) & 0xFF;
  const uint32_t front24 = front & 0xFFFFFFu;
  dir = (dir + (act == kLeft ? 3 : (act == kRight ? 1 : 0))) & 3;
  const bool walk = act == kForward && (type == kEmpty || type == kGoal || type == kLava ||
                                        (type == kDoor && state == kOpen));
  x = walk ? fx : x;
  y = walk ? fy : y;
  const bool pick = act == kPickup && carry == kCellEmpty && (type == kKey || type == kBall || type == kBox);
  const bool drop = act == kDrop && carry != kCellEmpty && type == kEmpty;
  const bool door = act == kToggle && type == kDoor;
  const bool unlock = door && state == kLocked && (carry & 0xFF) == kKey && ((carry >> 8) & 0xFF) == colour;
  const bool flip = door && state != kLocked;
  const uint32_t door_open = kDoor | (colour << 8) | (kOpen << 16);
  const uint32_t door_flipped = kDoor | (colour << 8) | ((state == kOpen ? kClosed : kOpen) << 16);
  ActResult r;
  r.new_front = pick ? kCellEmpty : (drop ? carry : (unlock ? door_open : (flip ? door_flipped : front24)));
  r.front_changed = pick || drop || unlock || flip;
  r.penalty = act == kForward && type == kLava;
  r.goal = act == kForward && type == kGoal;
  r.terminated = r.goal || r.penalty;
  carry = pick ? front24 : (drop ? kCellEmpty : carry);
  return r;
}

// ---------------------------------------------------------------------------
// Transition system of Dynamic-Obstacles (Table "systems"; Fig. 1): every
// ball, in list order, moves to a uniformly drawn empty cell of the 8
// around it that the agent does not occupy (the k-th in row-major order,
// k = u(count) of its word), or stays if there is none.  Ball b's word:
// key = seed, counter (rng_id, call, b / 4, 2), lane b % 4.  Cells: the
// grid accessor reads "is empty" and writes a ball or an empty cell.  List
// entries off the interior (only a malformed state has them) do not move.
// ---------------------------------------------------------------------------
// position of the k-th (0-based) set bit of an 8-bit m, k < popcount(m):
// halve the search range three times instead of clearing k bits one by one
__device__ __forceinline__ uint32_t kth_bit8(uint32_t m, uint32_t k) {
  uint32_t base = 0, p = (uint32_t)__builtin_popcount(m & 15u);
  const bool hi4 = k >= p;
  k -= hi4 ? p : 0u;
  m = hi4 ? m >> 4 : m;
  base += hi4 ? 4u : 0u;
  p = (uint32_t)__builtin_popcount(m & 3u);
  const bool hi2 = k >= p;
  k -= hi2 ? p : 0u;
  m = hi2 ? m >> 2 : m;
  base += hi2 ? 2u : 0u;
  return base + ((k >= (m & 1u)) ? 1u : 0u);
}

template <class Grid>
__device__ __forceinline__ void move_obstacles(const Grid& g, int n, int ax, int ay, uint32_t (&ob)[4],
                                               uint2 seed, uint32_t rng_id, uint32_t call) {
  uint4 blk = make_uint4(0, 0, 0, 0);
#pragma unroll
  for (int b = 0; b < kMaxObst; ++b) {
    if (b < n) {
      if ((b & 3) == 0) blk = philox10(make_uint4(rng_id, call, (uint32_t)(b >> 2), 2u), seed);
      const uint32_t word = pick4(blk, (uint32_t)(b & 3));
      const uint32_t pos = obst_at(ob, b);
      const int bx = (int)(pos & 0xFF), by = (int)(pos >> 8);
      // an entry off the interior (a malformed state) is left alone, so no
      // access ever leaves the env's grid
      const bool inside = bx >= 1 && by >= 1 && bx <= g.S - 2 && by <= g.S - 2;
      uint32_t mask = 0;   // bit i: neighbour i (row-major, the ball's own cell skipped) is empty
      if (inside) mask = g.free8(bx, by);
      // the agent's cell is never a destination
      const uint32_t ac = (uint32_t)(3 * (ay - by + 1) + (ax - bx + 1));
      if ((unsigned)(ax - bx + 1) < 3u && (unsigned)(ay - by + 1) < 3u && ac != 4u)
        mask &= ~(1u << (ac - (ac > 4u)));
      if (mask) {
        const uint32_t i = kth_bit8(mask, bounded(word, (uint32_t)__builtin_popcount(mask)));
        const uint32_t cell = i + (i >= 4u);   // 0..8 without the centre
        const int dx = (int)(cell % 3u) - 1, dy = (int)(cell / 3u) - 1;
        g.put_empty(bx, by);
        g.put_ball(bx + dx, by + dy);
        obst_set(ob, b, (uint32_t)(bx + dx), (uint32_t)(by + dy));
      }
    }
  }
}

// Reward of Eq. (1) in the time-discounted form 1 - 0.9 * (t / T), t after
// the step, as three IEEE fp32 operations; reward_mode 1: unit reward.
__device__ __forceinline__ float goal_reward(int32_t t, int32_t T, int32_t mode) {
  if (mode == 1) return 1.0f;
  const float q = __fdiv_rn((float)t, (float)T);
  const float p = __fmul_rn(0.9f, q);
  return __fsub_rn(1.0f, p);
}

// Reward of a step: -1 for walking into lava (R2 of Table "envs") or, in
// Dynamic-Obstacles, for stepping forward at a ball or wall (R3), in both
// modes; the goal reward on reaching the goal; else 0.
__device__ __forceinline__ float step_reward(const ActResult& r, int32_t t, int32_t T, int32_t mode) {
  return r.penalty ? -1.0f : (r.goal ? goal_reward(t, T, mode) : 0.0f);
}

// GoToDoor's rules on top of the intervention (on_door_done of Tables
// "rewards" and "terminations"): the done action (any value >= 6) with the
// mission's door directly ahead achieves the task; toggling ends the
// episode with reward 0.  mission = the target door's colour.
__device__ __forceinline__ void gotodoor_rules(ActResult& r, uint32_t act, uint32_t front, uint32_t mission) {
  const bool done_at = act >= 6u && (front & 0xFF) == kDoor && ((front >> 8) & 0xFF) == mission;
  r.goal = r.goal || done_at;
  r.terminated = r.terminated || done_at || act == kToggle;
}

// the mission reported with every record: GoToDoor's target colour, else 0xFF
__device__ __forceinline__ uint32_t mission_of(uint32_t fam, uint32_t ob0) {
  return fam == kFamGoToDoor ? (ob0 & 0xFFu) : 0xFFu;
}

// ---------------------------------------------------------------------------
// Observation O(s) (Table "observations", symbolic_first_person, R = 7):
// the 7x7 view ahead of the agent, agent at view column 3 of row 6; walls
// and non-open doors block sight.  Per view row the visible cells are the
// seeds plus the see-through runs that touch a see-through seed, widened
// by one cell on each side; the next row's seeds are the three cells ahead
// of every visible see-through cell.  This is MiniGrid's two-pass rule in
// bit-parallel form, the run fills being carry propagations.
// ---------------------------------------------------------------------------
// Row masks are kept in a dual form: the 7 column bits in bits 0-6 and the
// same bits reversed in bits 25-31.  One add then fills runs towards higher
// columns in the low half and towards lower columns in the high half (the
// carry out of bit 6 dies in the empty bit 7, that of bit 31 leaves the
// word), and one bit reversal merges the two directions.
__device__ __forceinline__ uint32_t visible_row(uint32_t seeds2, uint32_t see, uint32_t& next2) {
  const uint32_t p2 = see | __builtin_bitreverse32(see);
  const uint32_t g2 = seeds2 & p2;
  const uint32_t fill = (((p2 + g2) ^ p2) | g2) & p2;
  const uint32_t run2 = fill | __builtin_bitreverse32(fill);
  next2 = (run2 | (run2 << 1) | (run2 >> 1)) & 0xFE00007Fu;
  return seeds2 | next2;
}

// Computes the lane's observation obs[j][i][c] (147 bytes) as the 38 words
// u[0..37] it occupies once placed at byte 147 * slot of a record stage
// (slot = the lane's position in the staged group; slot 0 starts a group).
// rows.load_all(c) fills c[j][i] with the triple of view cell (i, j) and, when
// it is see-through, bit 31 - i set (no other bit of the top byte).  Lanes with valid == false produce zeros (their
// loader must still be safe to call).
//
// Records are realigned to their byte offset with byte permutes.  A word
// shared by two neighbouring records belongs to the higher one: u[0] of a
// record starting mid-word already holds the lower record's tail, received
// by a cross-lane shuffle; store_words writes exactly the words a record
// owns.
template <bool kCat, class Rows>
__device__ __forceinline__ void observe_words(const Rows& rows, uint32_t carry, bool valid, int slot,
                                              uint32_t (&u)[kObsWords + 1]) {
  constexpr int kBytes = kCat ? kCatBytes : kObsBytes;
  constexpr int kWords = kCat ? kCatWords : kObsWords;
  const uint32_t m = (uint32_t)(kBytes * slot) & 3u;
  const uint32_t realign = 0x07060504u - m * 0x01010101u;

  // all 49 reads first: they are independent and stay in flight together
  uint32_t cells[kView][kView];
  rows.load_all(cells);

  uint32_t seeds = valid ? ((1u << 3) | (1u << 28)) : 0u;   // column 3, dual form
  // masked first cells of the row processed before (row j + 1); zero past
  // the record's end
  uint32_t later[3] = {0u, 0u, 0u};
  uint32_t w_hi = 0;          // record word d + 1 (zero past the end)
#pragma unroll
  for (int j = kView - 1; j >= 0; --j) {
    uint32_t (&c)[kView] = cells[j];
    // see-through bits: cell i carries its flag at bit 31 - i, so the row's
    // flags are one OR away, already in the high half of the dual form
    const uint32_t see = ((c[0] | c[1] | c[2]) | (c[3] | c[4] | c[5]) | c[6]) & kSeeBits;
    uint32_t next;
    const uint32_t vis = visible_row(seeds, see, next);
    seeds = next;
#pragma unroll
    for (int i = 0; i < kView; ++i) c[i] &= (uint32_t)(((int32_t)(vis << (31 - i))) >> 31);
    if (j == kView - 1) c[3] = valid ? carry : 0u;   // the agent's cell shows what it carries
#pragma unroll
    for (int d = kWords - 1; d >= 0; --d) {
      uint32_t wd;
      if (kCat) {
        // word d holds the types of cells 4d .. 4d + 3 (byte b = cell b)
        const int k = 4 * d;
        if (k / kView != j) continue;
        const int i = k - kView * j;
        const uint32_t c0 = c[i];
        const uint32_t c1 = i + 1 < kView ? c[i + 1] : later[i + 1 - kView];
        const uint32_t c2 = i + 2 < kView ? c[i + 2] : later[i + 2 - kView];
        const uint32_t c3 = i + 3 < kView ? c[i + 3] : later[i + 3 - kView];
        wd = __builtin_amdgcn_perm(__builtin_amdgcn_perm(c3, c2, 0x0C0C0400u),
                                   __builtin_amdgcn_perm(c1, c0, 0x0C0C0400u), 0x05040100u);
      } else {
        // word d spans cells 4d/3 and 4d/3 + 1 (byte b belongs to cell b / 3)
        const int k = (4 * d) / 3;
        if (k / kView != j) continue;
        const int i = k - kView * j, off = (4 * d) % 3;
        const uint32_t sel = off == 0 ? 0x04020100u : (off == 1 ? 0x05040201u : 0x06050402u);
        wd = __builtin_amdgcn_perm(i + 1 < kView ? c[i + 1] : later[0], c[i], sel);
      }
      u[d + 1] = __builtin_amdgcn_perm(w_hi, wd, realign);
      w_hi = wd;
    }
    later[0] = c[0];
    later[1] = c[1];
    later[2] = c[2];
  }
  u[0] = __builtin_amdgcn_perm(w_hi, 0u, realign);
  // the word a record shares with the next one (the one holding the next
  // record's first byte): symbolic u[36] when the record starts on a word
  // boundary, u[37] when it starts two or three bytes in; categorical u[12]
  const uint32_t tail = kCat ? u[kCatWords - 1] : (m == 0 ? u[kObsWords - 1] : u[kObsWords]);
  const uint32_t lower_tail = (uint32_t)__shfl_up((int)tail, 1, kWave);
  if (m != 0) u[0] |= lower_tail;
}

// Writes the words a record owns (see observe_words) at stage + bytes * slot:
// all but the word holding the next record's first byte, which that record
// writes (symbolic: the next record starts inside word 36 unless m == 1 puts
// it at word 37; categorical: inside word 12 unless m == 3).
template <bool kCat>
__device__ __forceinline__ void store_words(uint8_t* stage, int slot, const uint32_t (&u)[kObsWords + 1]) {
  constexpr int kBytes = kCat ? kCatBytes : kObsBytes;
  constexpr int kWords = kCat ? kCatWords : kObsWords;
  const uint32_t s = (uint32_t)(kBytes * slot);
  const uint32_t m = s & 3u;
  uint32_t* base = reinterpret_cast<uint32_t*>(stage) + (s >> 2);
#pragma unroll
  for (int q = 0; q < kWords - 1; ++q) base[q] = u[q];
  if (kCat ? m == 3 : m != 0) base[kWords - 1] = u[kWords - 1];
}

// Both kernels' workgroups are single waves and all the data its lanes
// exchange lives in LDS, whose operations a wave performs in issue order: a
// wavefront-scope fence (no wait instruction) plus a compiler barrier is
// enough to make one lane's LDS writes visible to the others' later reads.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Copies the first `bytes` (1 <= bytes <= kMaxBytes) staged bytes to dst.
// To a 16-byte aligned dst the whole 16-byte chunks go as vector stores
// (all of a lane's LDS reads issued before its stores, so the reads are in
// flight together) and the last bytes % 16 bytes one by one; otherwise
// every byte goes alone.
template <int kMaxBytes>
__device__ __forceinline__ void copy_piece(const uint8_t* stage, uint8_t* dst, int bytes, int lane) {
  constexpr int kMaxChunks = (kMaxBytes + 15) / 16;
  constexpr int kPerLane = (kMaxChunks + kWave - 1) / kWave;
  if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
    const u32x4* src = reinterpret_cast<const u32x4*>(stage);
    u32x4* out = reinterpret_cast<u32x4*>(dst);
    const int n = bytes >> 4;
    if (n > 0) {
      // Reads clamp to the last chunk so they need no branch.
      u32x4 v[kPerLane];
#pragma unroll
      for (int i = 0; i < kPerLane; ++i) v[i] = src[min(lane + i * kWave, n - 1)];
#pragma unroll
      for (int i = 0; i < kPerLane; ++i) {
        const int c = lane + i * kWave;
        if (c < n) __builtin_nontemporal_store(v[i], out + c);
      }
    }
    if (lane < (bytes & 15)) dst[16 * n + lane] = stage[16 * n + lane];
  } else {
    for (int b = lane; b < bytes; b += kWave) dst[b] = stage[b];
  }
}

// Copies n_envs staged records of kBytes bytes (1 <= n_envs <= kMaxEnvs) to dst.
template <int kMaxEnvs, int kBytes>
__device__ __forceinline__ void copy_out(const uint8_t* stage, uint8_t* dst, int n_envs, int lane) {
  copy_piece<kMaxEnvs * kBytes>(stage, dst, n_envs * kBytes, lane);
}

// ---------------------------------------------------------------------------
// Whole-grid observations (Table "observations": symbolic [S][S][3] and
// categorical [S][S]), MiniGrid's fully observed encoding: every cell's
// triple (or type) with the agent drawn over its own cell as (10, red,
// heading).  A wave's records are contiguous in the output row, exactly like
// its envs' grids, so the wave writes them as one byte range [0, n): window
// by window, the lanes fill the LDS stage a word at a time (fill(o) returns
// output bytes o..o+3; o may fall outside [0, n) at the window edges, where
// the bytes are never stored), every lane then writes its agent's bytes over
// its cell, and the window leaves as 16-byte aligned stores; bytes outside
// [0, n) belong to neighbouring waves' records and are left alone.
// ---------------------------------------------------------------------------
constexpr uint32_t kAgent = 10;

template <int kWin, class Fill>
__device__ __forceinline__ void emit_grids(uint8_t* dst, int64_t n, uint8_t* stage, int lane, bool has_agent,
                                           int64_t agent_o, uint32_t agent_bytes, int agent_len,
                                           const Fill& fill) {
  static_assert(kWin % 16 == 0, "stage windows are whole 16-byte chunks");
  const uintptr_t d0 = reinterpret_cast<uintptr_t>(dst), d1 = d0 + (uintptr_t)n;
  uint32_t* words = reinterpret_cast<uint32_t*>(stage);
  // windows start on 64-byte boundaries of the output (kWin is a multiple
  // of 64), so every store instruction covers whole 64-byte units of HBM
  static_assert(kWin % 64 == 0, "windows keep the 64-byte alignment");
  for (uintptr_t A = d0 & ~(uintptr_t)63; A < d1; A += kWin) {
    const int win = (int)min((uintptr_t)kWin, (d1 - A + 15) & ~(uintptr_t)15);
    const int64_t rel = (int64_t)A - (int64_t)d0;   // output byte of stage byte 0, >= -63
    for (int q = lane; q < (win >> 2); q += kWave) words[q] = fill(rel + 4 * q);
    wave_sync();
    if (has_agent) {
      for (int k = 0; k < agent_len; ++k) {
        const int64_t p = agent_o + k - rel;
        if (p >= 0 && p < win) stage[p] = (uint8_t)(agent_bytes >> (8 * k));
      }
    }
    wave_sync();
    for (int c = lane; c < (win >> 4); c += kWave) {
      const uintptr_t a = A + 16 * (uintptr_t)c;
      if (a >= d0 && a + 16 <= d1) {
        __builtin_nontemporal_store(reinterpret_cast<const u32x4*>(stage)[c], reinterpret_cast<u32x4*>(a));
      } else {
        for (int b = 0; b < 16; ++b)
          if (a + b >= d0 && a + b < d1) reinterpret_cast<uint8_t*>(a)[b] = stage[16 * c + b];
      }
    }
    wave_sync();
  }
}

// Fill of symbolic records from the HBM grids (the plain kernel): output
// byte o is byte o of the wave's grid block of n bytes.
struct FillHbmSymbolic {
  const uint8_t* src;
  int64_t n;
  __device__ __forceinline__ uint32_t operator()(int64_t o) const {
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (o + k >= 0 && o + k < n) w |= (uint32_t)src[o + k] << (8 * k);
    return w;
  }
};

// Categorical records from the HBM grids: output byte o is the type channel
// of cell o of the wave's block of n cells.
struct FillHbmCategorical {
  const uint8_t* src;
  int64_t n;
  __device__ __forceinline__ uint32_t operator()(int64_t o) const {
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (o + k >= 0 && o + k < n) w |= (uint32_t)src[3 * (o + k)] << (8 * k);
    return w;
  }
};

// ---------------------------------------------------------------------------
// Plain kernel
// ---------------------------------------------------------------------------
// Cell (x, y) for view column i: the triple, plus bit 31 - i if see-through.
struct HbmCells {
  const uint8_t* g;
  int S;
  __device__ __forceinline__ uint32_t operator()(int x, int y, int i) const {
    if ((unsigned)x >= (unsigned)S || (unsigned)y >= (unsigned)S) return kCellWall;
    const uint8_t* p = g + 3 * (y * S + x);
    const uint32_t tri = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
    return tri | (see_through(tri) >> i);
  }
};

// The 7x7 view straight from the HBM grid, cells outside it read as walls.
// Whatever the heading, the view covers a 7x7 square of the world: 7 grid
// rows of 7 consecutive cells, i.e. 21 contiguous bytes each.  A row is
// read as the 24 bytes from its dword-aligned start (one 16-byte and one
// 8-byte load) instead of 21 byte loads; near the grid's first and last
// bytes the row falls back to single dwords, each read only if it holds a
// byte of the env's grid.  The square is then turned to the view's
// orientation by selects on the heading.
struct HbmWindow {
  const uint8_t* g;
  int S;   // 0: every cell reads as a wall
  int ax, ay, dir;
  __device__ __forceinline__ void load_all(uint32_t (&c)[kView][kView]) const {
    // top-left world cell of the square
    const int x0 = dir == 0 ? ax : (dir == 2 ? ax - 6 : ax - 3);
    const int y0 = dir == 3 ? ay - 6 : (dir == 1 ? ay : ay - 3);
    const uintptr_t gb = reinterpret_cast<uintptr_t>(g);
    const uintptr_t lo = gb & ~(uintptr_t)3, hi = (gb + 3 * (uintptr_t)(S * S) + 3) & ~(uintptr_t)3;
    uint32_t w[kView][6];
#pragma unroll
    for (int r = 0; r < kView; ++r) {
      const int yy = y0 + r;
#pragma unroll
      for (int d = 0; d < 6; ++d) w[r][d] = 0u;
      if ((unsigned)yy < (unsigned)S) {
        const uintptr_t a = (uintptr_t)((intptr_t)gb + 3 * (intptr_t)(yy * S + x0)) & ~(uintptr_t)3;
        if (a >= lo && a + 24 <= hi) {
          const uint32_t* q = reinterpret_cast<const uint32_t*>(a);
          const u32x4 v4 = *reinterpret_cast<const u32x4*>(q);
          const uint2 v2 = *reinterpret_cast<const uint2*>(q + 4);
          w[r][0] = v4.x; w[r][1] = v4.y; w[r][2] = v4.z; w[r][3] = v4.w;
          w[r][4] = v2.x; w[r][5] = v2.y;
        } else {
#pragma unroll
          for (int d = 0; d < 6; ++d)
            if (a + 4 * d >= lo && a + 4 * d < hi) w[r][d] = reinterpret_cast<const uint32_t*>(a)[d];
        }
      }
    }
    // world cell (x0 + k, y0 + r), with its see-through flag at bit 31
    uint32_t W[kView][kView];
#pragma unroll
    for (int r = 0; r < kView; ++r) {
      const int yy = y0 + r;
      const uint32_t rb = (uint32_t)((uintptr_t)((intptr_t)gb + 3 * (intptr_t)(yy * S + x0)) & 3);
      uint32_t b[6];
#pragma unroll
      for (int d = 0; d < 5; ++d) b[d] = __builtin_amdgcn_alignbyte(w[r][d + 1], w[r][d], rb);
      b[5] = w[r][5] >> (8 * rb);
#pragma unroll
      for (int k = 0; k < kView; ++k) {
        const int o = 3 * k, d = o >> 2, off = o & 3;
        const uint32_t tri = (__builtin_amdgcn_alignbyte(b[d + 1], b[d], (uint32_t)off)) & 0xFFFFFFu;
        const bool in = (unsigned)yy < (unsigned)S && (unsigned)(x0 + k) < (unsigned)S;
        W[r][k] = in ? tri | see_through(tri) : kCellWall;
      }
    }
    // view cell (i, j) = world a + (i - 3) right + (6 - j) ahead
#pragma unroll
    for (int j = 0; j < kView; ++j)
#pragma unroll
      for (int i = 0; i < kView; ++i) {
        uint32_t v = W[j][i];                              // north
        v = dir == 0 ? W[i][6 - j] : v;                    // east
        v = dir == 1 ? W[6 - j][6 - i] : v;                // south
        v = dir == 2 ? W[6 - i][j] : v;                    // west
        c[j][i] = (v & ~kSeeBit) | ((v & kSeeBit) >> i);
      }
  }
};

// The plain kernel's view, read before the action is applied.  The step can
// only end in one of two 7x7 squares: a turn ends in the new heading's
// square; forward ends in the current square or in the one a cell ahead;
// every other action (and a reset) keeps the current square.  Their union is
// the final heading's square extended by one cell along that heading, at
// most 8 grid rows of 8 cells, and it holds the cell ahead as well.  Reading
// it as soon as the action is known puts the cell ahead and the view in one
// round trip to HBM instead of two dependent ones.
//
// Region cell (k, r) is world cell (X0 + k, Y0 + r).  Heading east the region
// starts at the agent's column, west 7 cells behind it; south at the agent's
// row, north 7 rows above it; across the heading it spans the square's 7
// cells.  The final square starts at offset m along the heading: east and
// south m = 1 when the agent moved, west and north m = 0 when it moved.
struct HbmSpan {
  uint32_t w[8][7];   // row r: the 28 bytes from the dword-aligned start of cell (X0, Y0 + r)
  uintptr_t gb;
  int S, X0, Y0, dir;

  // dir: the heading the step ends with; rows outside the grid and the
  // eighth row of a horizontal heading are not read
  __device__ __forceinline__ void load(const uint8_t* g, int S_, int ax, int ay, int dir_) {
    gb = reinterpret_cast<uintptr_t>(g);
    S = S_;
    dir = dir_;
    X0 = dir == 0 ? ax : (dir == 2 ? ax - 7 : ax - 3);
    Y0 = dir == 1 ? ay : (dir == 3 ? ay - 7 : ay - 3);
    const bool vert = (dir & 1) != 0;
    const uintptr_t lo = gb & ~(uintptr_t)3, hi = (gb + 3 * (uintptr_t)(S * S) + 3) & ~(uintptr_t)3;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int yy = Y0 + r;
#pragma unroll
      for (int d = 0; d < 7; ++d) w[r][d] = 0u;
      if ((unsigned)yy < (unsigned)S && (r < 7 || vert)) {
        const uintptr_t a = (uintptr_t)((intptr_t)gb + 3 * (intptr_t)(yy * S + X0)) & ~(uintptr_t)3;
        if (a >= lo && a + 28 <= hi) {
          const u32x4 v4 = *reinterpret_cast<const u32x4*>(a);
          const uint32_t* q = reinterpret_cast<const uint32_t*>(a + 16);
          w[r][0] = v4.x; w[r][1] = v4.y; w[r][2] = v4.z; w[r][3] = v4.w;
          w[r][4] = q[0]; w[r][5] = q[1]; w[r][6] = q[2];
        } else {
#pragma unroll
          for (int d = 0; d < 7; ++d)
            if (a + 4 * d >= lo && a + 4 * d < hi) w[r][d] = reinterpret_cast<const uint32_t*>(a)[d];
        }
      }
    }
  }

  // the triple of region cell (k, r); a cell outside the grid reads as
  // whatever the loaded bytes hold there (bytes of the grid's other rows, up
  // to 3 bytes of a neighbouring env's grid in the dwords at the grid's two
  // ends, or zeros for rows that were not read)
  __device__ __forceinline__ uint32_t cell(int k, int r) const {
    const int yy = Y0 + r;
    const uint32_t rb = (uint32_t)((uintptr_t)((intptr_t)gb + 3 * (intptr_t)(yy * S + X0)) & 3);
    const int o = 3 * k, d = o >> 2, off = o & 3;
    const uint32_t b0 = __builtin_amdgcn_alignbyte(w[r][d + 1], w[r][d], rb);
    const uint32_t b1 = d + 2 < 7 ? __builtin_amdgcn_alignbyte(w[r][d + 2], w[r][d + 1], rb) : w[r][d + 1] >> (8 * rb);
    return __builtin_amdgcn_alignbyte(b1, b0, (uint32_t)off) & 0xFFFFFFu;
  }

  // the cell ahead of the agent before it moves (heading dir, no turn)
  __device__ __forceinline__ uint32_t front() const {
    return dir == 0 ? cell(1, 3) : (dir == 1 ? cell(3, 1) : (dir == 2 ? cell(6, 3) : cell(3, 6)));
  }

  // c[j][i] as for observe_words, for the square at offset m along the
  // heading; `patch` replaces the cell ahead of the unmoved agent (a
  // pickup, drop or toggle, which neither move nor turn it).  Cells outside
  // the grid are not masked: whenever the grid's outer ring is opaque (walls
  // and closed or locked doors) sight never crosses it, so none of them is
  // ever visible.  Only a door on the ring toggled open breaks that, and
  // such a step reads its view bounds-checked instead.
  __device__ __forceinline__ void view(bool moved, bool patch, uint32_t new_front,
                                       uint32_t (&c)[kView][kView]) const {
    const bool vert = (dir & 1) != 0;
    const bool m = moved != (dir >= 2);
    uint32_t R[8][8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int k = 0; k < 8; ++k) R[r][k] = (r == 7 && k == 7) ? 0u : cell(k, r);
    const uint32_t nf = new_front;
    R[3][1] = patch && dir == 0 ? nf : R[3][1];
    R[1][3] = patch && dir == 1 ? nf : R[1][3];
    R[3][6] = patch && dir == 2 ? nf : R[3][6];
    R[6][3] = patch && dir == 3 ? nf : R[6][3];
    // world cell (X0 + k, Y0 + r) of the final square, offset applied
    uint32_t W[kView][kView];
#pragma unroll
    for (int r = 0; r < kView; ++r)
#pragma unroll
      for (int k = 0; k < kView; ++k) W[r][k] = m ? (vert ? R[r + 1][k] : R[r][k + 1]) : R[r][k];
    // view cell (i, j) = world a + (i - 3) right + (6 - j) ahead
#pragma unroll
    for (int j = 0; j < kView; ++j)
#pragma unroll
      for (int i = 0; i < kView; ++i) {
        uint32_t v = W[j][i];                              // north
        v = dir == 0 ? W[i][6 - j] : v;                    // east
        v = dir == 1 ? W[6 - j][6 - i] : v;                // south
        v = dir == 2 ? W[6 - i][j] : v;                    // west
        c[j][i] = v | (see_through(v) >> i);
      }
  }
};

// A view computed beforehand, handed to observe_words.
struct ViewCells {
  const uint32_t (&c)[kView][kView];
  __device__ __forceinline__ void load_all(uint32_t (&o)[kView][kView]) const {
#pragma unroll
    for (int j = 0; j < kView; ++j)
#pragma unroll
      for (int i = 0; i < kView; ++i) o[j][i] = c[j][i];
  }
};

// View rows straight from the HBM grid, cells outside it read as walls.
struct HbmRows {
  HbmCells cells;
  int ax, ay, fx, fy;
  __device__ __forceinline__ void load(int j, uint32_t (&c)[kView]) const {
    const int rx = -fy, ry = fx;
    const int bx = ax - 3 * rx + (6 - j) * fx, by = ay - 3 * ry + (6 - j) * fy;
#pragma unroll
    for (int i = 0; i < kView; ++i) c[i] = cells(bx + i * rx, by + i * ry, i);
  }
  __device__ __forceinline__ void load_all(uint32_t (&c)[kView][kView]) const {
#pragma unroll
    for (int j = kView - 1; j >= 0; --j) load(j, c[j]);
  }
};

__device__ __forceinline__ void store_triple(uint8_t* p, uint32_t tri) {
  p[0] = (uint8_t)tri;
  p[1] = (uint8_t)(tri >> 8);
  p[2] = (uint8_t)(tri >> 16);
}

// Grid accessors for the obstacle transition: HBM triples, LDS codes.
struct HbmGrid {
  uint8_t* g;
  int S;
  // the 8 cells around interior cell (x, y), row-major, as bits: set = empty
  __device__ __forceinline__ uint32_t free8(int x, int y) const {
    const uint8_t* p = g + 3 * ((y - 1) * S + (x - 1));
    const uint8_t* q = p + 3 * S;
    const uint8_t* r = q + 3 * S;
    return (p[0] == kEmpty ? 1u : 0u) | (p[3] == kEmpty ? 2u : 0u) | (p[6] == kEmpty ? 4u : 0u) |
           (q[0] == kEmpty ? 8u : 0u) | (q[6] == kEmpty ? 16u : 0u) | (r[0] == kEmpty ? 32u : 0u) |
           (r[3] == kEmpty ? 64u : 0u) | (r[6] == kEmpty ? 128u : 0u);
  }
  __device__ __forceinline__ void put_empty(int x, int y) const { store_triple(g + 3 * (y * S + x), kCellEmpty); }
  __device__ __forceinline__ void put_ball(int x, int y) const { store_triple(g + 3 * (y * S + x), kCellBall); }
};

struct PlainArgs {
  EnvTables env;
  StateBufs st;
  const uint8_t* actions;
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

  uint32_t fam = 0, meta = 0;
  int S = 5, T = 1, x = 1, y = 1, dir = 0, t = 0;
  uint32_t carry = kCellEmpty, episode = 0, rid = 0, calls = 0;
  bool done_prev = false;
  uint2 seed = make_uint2(0, 0);
  uint8_t* g = a.st.grid;
  uint64_t goff = 0;
  uint32_t ob[4] = {~0u, ~0u, ~0u, ~0u};
  if (active) {
    meta = a.env.meta[e];
    fam = meta & 0xFF;
    S = (int)((meta >> 8) & 0xFF);
    T = a.env.max_steps[e];
    seed = a.env.seed[e];
    rid = a.env.rng_id[e];
    goff = a.env.grid_off[e];
    g = a.st.grid + goff;
    if (!a.reset_all) {
      x = a.st.x[e];
      y = a.st.y[e];
      dir = a.st.dir[e];
      t = a.st.t[e];
      carry = (uint32_t)a.st.carry[e];
      episode = a.st.episode[e];
      done_prev = a.st.done_prev[e] != 0;
      calls = a.st.calls[e];
      if (fam == kFamDynObs || fam == kFamGoToDoor) {   // the balls, or the mission
        const uint4 o4 = *reinterpret_cast<const uint4*>(a.st.obst + 16 * (size_t)e);
        ob[0] = o4.x; ob[1] = o4.y; ob[2] = o4.z; ob[3] = o4.w;
      }
    }
  }
  const bool do_reset = active && (a.reset_all || done_prev);
  Layout L{};
  if (do_reset) {
    episode = a.reset_all ? 0u : episode + 1u;
    L = make_layout(meta, seed, rid, episode);
    x = L.ax;
    y = L.ay;
    dir = L.dir;
    t = 0;
    carry = kCellEmpty;
#pragma unroll
    for (int i = 0; i < 4; ++i) ob[i] = L.ob[i];
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

  uint32_t act = 0;
  if (active && !do_reset) {
    if (a.actions) {
      act = a.actions[e];
    } else {
      act = bounded(pick4(policy_block(seed, rid, calls), calls & 3u), 7u);
    }
  }
  // The first-person modes read the view as soon as the action is known
  // (HbmSpan), the cell ahead included.  Dynamic-Obstacles envs, whose
  // balls move before the action applies, read the cell ahead and the view
  // from HBM afterwards instead, and so does every env when the records are
  // whole grids (copied from the grids) or not written at all.
  const bool span_view = a.out.obs != nullptr && a.env.obs_mode < 2;
  HbmSpan span;
  if (span_view) {
    const int dir_f = do_reset ? dir : (dir + (act == kLeft ? 3 : (act == kRight ? 1 : 0))) & 3;
    span.load(g, active && fam != kFamDynObs ? S : 0, x, y, dir_f);
  }

  float reward = 0.0f;
  uint32_t flags = 0, act_rec = kActionNone;
  bool moved = false, patch = false, edge_view = false;
  uint32_t new_front = 0;
  if (active && !do_reset) {
    const int fx = x + dir_dx(dir), fy = y + dir_dy(dir);
    const HbmCells cells{g, S};
    const bool ahead_in_span = span_view && fam != kFamDynObs;
    uint32_t front;
    if (ahead_in_span) front = span.front();
    else front = cells(fx, fy, 0);
    bool blocked = false;
    if (fam == kFamDynObs) {
      // three actions; the cell ahead is judged before the balls move
      act = act > kForward ? kLeft : act;
      blocked = (front & 0xFF) != kEmpty && (front & 0xFF) != kGoal;
      move_obstacles(HbmGrid{g, S}, (int)((meta >> 16) & 0xFF), x, y, ob, seed, rid, calls);
      front = cells(fx, fy, 0);
    }
    const int x_was = x, y_was = y;
    ActResult r = intervene(act, x, y, dir, carry, front, fx, fy);
    moved = x != x_was || y != y_was;
    r.penalty = r.penalty || (blocked && act == kForward);
    r.terminated = r.terminated || r.penalty;
    if (fam == kFamGoToDoor) gotodoor_rules(r, act, front, ob[0] & 0xFFu);
    if (r.front_changed) store_triple(g + 3 * (fy * S + fx), r.new_front);
    patch = r.front_changed;
    new_front = r.new_front;
    edge_view = fam == kFamGoToDoor && r.front_changed;   // a door toggled, possibly on the outer ring
    t += 1;
    const bool trunc = t >= T;
    reward = step_reward(r, t, T, a.env.reward_mode);
    flags = (r.terminated ? kFlagTerminated : 0u) | (trunc ? kFlagTruncated : 0u);
    done_prev = r.terminated || trunc;
    act_rec = act & 0xFF;
  } else if (do_reset) {
    flags = kFlagFirst;
    done_prev = false;
  }

  const size_t rowN = (size_t)a.row * (size_t)N;
  if (a.out.obs && a.env.obs_mode >= 2) {
    // whole-grid records: the step's grid writes by every lane (resets,
    // doors, keys, balls) must be visible before the wave copies the grids
    __threadfence_block();
    __syncthreads();
    const uint64_t G0 = (uint64_t)__shfl((long long)goff, 0, kWave);
    const uint64_t end = active ? goff + 3ull * (uint64_t)(S * S) : 0ull;
    const int64_t n = (int64_t)((uint64_t)__shfl((long long)end, n_here - 1, kWave) - G0);
    const int64_t cell = (int64_t)(goff - G0) / 3 + y * S + x;   // the agent's cell in the block
    const uint8_t* src = a.st.grid + G0;
    uint8_t* dst = a.out.obs + (size_t)a.row * a.out.obs_row;
    if (a.env.obs_mode == 3)
      emit_grids<kStageBytes>(dst + G0 / 3, n / 3, stage, lane, active, cell, kAgent, 1,
                              FillHbmCategorical{src, n / 3});
    else
      emit_grids<kStageBytes>(dst + G0, n, stage, lane, active, 3 * cell, kAgent | ((uint32_t)dir << 16), 3,
                              FillHbmSymbolic{src, n});
  } else if (a.out.obs) {
    // inactive lanes read no cell (S = 0 above): every cell is a wall
    uint32_t u[kObsWords + 1];
    uint32_t view[kView][kView];
    span.view(moved, patch, new_front, view);
    // balls that moved, or a door on the ring toggled open: read the view
    // again, bounds-checked, from the grid as the step left it
    if (fam == kFamDynObs || edge_view) HbmWindow{g, S, x, y, dir}.load_all(view);
    const ViewCells rows{view};
    if (a.env.obs_mode == 1) {
      observe_words<true>(rows, carry, active, lane, u);
      store_words<true>(stage, lane, u);
      __syncthreads();
      copy_out<kWave, kCatBytes>(stage, a.out.obs + (rowN + (size_t)e0) * kCatBytes, n_here, lane);
    } else {
      observe_words<false>(rows, carry, active, lane, u);
      store_words<false>(stage, lane, u);
      __syncthreads();
      copy_out<kWave, kObsBytes>(stage, a.out.obs + (rowN + (size_t)e0) * kObsBytes, n_here, lane);
    }
  }
  if (active && a.out.reward) {
    a.out.reward[rowN + e] = reward;
    a.out.flags[rowN + e] = (uint8_t)flags;
    a.out.action[rowN + e] = (uint8_t)act_rec;
    if (a.out.mission) a.out.mission[rowN + e] = (uint8_t)mission_of(fam, ob[0]);
  }
  if (active) {
    a.st.x[e] = x;
    a.st.y[e] = y;
    a.st.dir[e] = dir;
    a.st.t[e] = t;
    a.st.carry[e] = (int32_t)carry;
    a.st.episode[e] = episode;
    a.st.done_prev[e] = done_prev ? 1 : 0;
    a.st.calls[e] = a.reset_all ? 0u : calls + 1u;
    if (fam == kFamDynObs || do_reset)
      *reinterpret_cast<uint4*>(a.st.obst + 16 * (size_t)e) = make_uint4(ob[0], ob[1], ob[2], ob[3]);
  }
}

// ---------------------------------------------------------------------------
// Fused kernel
// ---------------------------------------------------------------------------
// One byte per cell in LDS: four times the cell's kind, i.e. the byte
// offset of its entry in 64-entry tables of triples, so a cell costs one byte
// read and one table read.  There is one table per view column i, whose
// entries carry the see-through flag at bit 31 - i.  Kinds: 0 empty;
// 1-6 wall, 7-12 goal, 13-18 key, 19-24 ball, 25-30 box by colour; 31-48
// door by state and colour; 49 lava; 50 anything else (read as unseen);
// 51-54 the agent by heading (whole-grid records only).
__device__ __forceinline__ uint32_t code_of(uint32_t tri) {
  const uint32_t type = tri & 0xFF, colour = (tri >> 8) & 0xFF, state = (tri >> 16) & 0xFF;
  // first kind of each type, as two 8-entry byte tables read with v_perm:
  // types 0-3 {50, 0, 1, 50}, 4-7 {31, 13, 19, 25}, 8-11 {7, 49, 50, 50}, 12-15 all 50
  const uint32_t lo = __builtin_amdgcn_perm(0x19130D1Fu, 0x32010032u, type & 7);
  const uint32_t hi = __builtin_amdgcn_perm(0x32323232u, 0x32323107u, type & 7);
  uint32_t kind = (type < 8 ? lo : hi) & 0xFF;
  kind = type > 15 ? 50u : kind;
  // walls, doors, keys, balls, boxes and goals come in colours; doors in states
  kind += ((0x1F4u >> (type & 15)) & 1u) ? colour : 0u;
  kind += type == kDoor ? 6u * state : 0u;
  return (kind << 2) & 0xFFu;
}

// kinds 51-54: the agent facing east, south, west, north; they exist only
// while whole-grid records are written
constexpr uint32_t kAgentKind = 51;

__device__ __forceinline__ uint32_t triple_of_kind(uint32_t kind) {
  uint32_t tri;
  if (kind == 0) tri = kCellEmpty;
  else if (kind <= 6) tri = kWall | ((kind - 1) << 8);
  else if (kind <= 12) tri = kGoal | ((kind - 7) << 8);
  else if (kind <= 18) tri = kKey | ((kind - 13) << 8);
  else if (kind <= 24) tri = kBall | ((kind - 19) << 8);
  else if (kind <= 30) tri = kBox | ((kind - 25) << 8);
  else if (kind <= 48) tri = kDoor | (((kind - 31) % 6) << 8) | (((kind - 31) / 6) << 16);
  else if (kind == 49) tri = 9;
  else if (kind >= kAgentKind && kind < kAgentKind + 4) return kAgent | ((kind - kAgentKind) << 16);
  else return 0;
  return tri | see_through(tri);
}

constexpr int kKinds = 64;

// code of cell (x, y) of a freshly generated layout (grey walls, green
// goal, key and locked door of the layout's colour, red lava); equals
// code_of(layout_cell(L, x, y)) without the general switch
__device__ __forceinline__ uint32_t layout_code(const Layout& L, int x, int y) {
  constexpr uint32_t kWallCode = 4 * (1 + kGrey), kGoalCode = 4 * (7 + kGreen), kLavaCode = 4 * 49;
  const int S = L.S;
  if (L.fam == kFamKeyCorridor) return code_of(keycorridor_cell(L, x, y));
  uint32_t code = 0;
  if (L.fam == kFamTwoRoom) {   // the family is uniform across the wave here
    code = (x == L.kx && y == L.ky) ? 4u * (13u + (uint32_t)L.colour) : code;
    code = x == L.a ? (y == L.b ? 4u * (31u + 6u * kLocked + (uint32_t)L.colour) : kWallCode) : code;
  } else if (L.fam == kFamFourRooms) {
    const int m = S / 2;
    code = (y == m && x != L.c && x != L.d) ? kWallCode : code;
    code = (x == m && y != L.a && y != L.b) ? kWallCode : code;
  } else if (L.fam == kFamLavaGap) {
    code = (x == L.a && y != L.b) ? kLavaCode : code;
  } else if (L.fam == kFamCrossings) {
    code = crossings_lava(L, x, y) ? kLavaCode : code;
  } else if (L.fam == kFamDistShift) {
    code = ((y == 1 || y == L.a) && x >= 3 && x <= S - 3) ? kLavaCode : code;
  } else if (L.fam == kFamDynObs) {
    code = is_ball(L, x, y) ? 4u * (19u + kBlue) : code;
  } else if (L.fam == kFamGoToDoor) {
    const int dc = gotodoor_door(L, x, y);
    const bool wall = x == 0 || y == 0 || x >= L.kx - 1 || y >= L.ky - 1;
    return dc >= 0 ? 4u * (31u + 6u * kClosed + (uint32_t)dc) : (wall ? kWallCode : 0u);
  }
  code = (x == L.gx && y == L.gy) ? kGoalCode : code;
  const bool border = x == 0 || y == 0 || x == S - 1 || y == S - 1;
  return border ? kWallCode : code;
}
// A view reaches at most 6 cells ahead and 3 to the side of an interior
// agent, i.e. at most 5 rows and 5 columns outside an S <= 32 grid: with
// row-major indexing that is within 5 * 32 + 5 = 165 bytes before or after
// the grid.  Such cells are never visible (the wall border blocks sight),
// so only their addresses must stay inside the allocation.
constexpr int kMargin = 192;

// dynamic LDS of a fused workgroup: the largest tile's grids plus both margins
__host__ __device__ inline size_t tile_lds_bytes(int32_t max_tile_cells) {
  const size_t b = 2 * (size_t)kMargin + (size_t)max_tile_cells;
  return (b + 15) & ~(size_t)15;
}

__device__ __forceinline__ uint32_t table_at(const uint32_t* table, uint32_t code4) {
  return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(table) + code4);
}

// View rows from the LDS code grid: the view's row and column steps are
// +-1 or +-S in the row-major grid, so each cell is one add away.  All 49
// codes are read before any table lookup, so the lookups wait on the code
// reads in bulk rather than one dependent pair at a time.
struct LdsRows {
  const uint32_t* table;
  const uint8_t* center;   // the agent's cell
  int R, F;                // linear steps to the agent's right and ahead
  __device__ __forceinline__ void load_all(uint32_t (&c)[kView][kView]) const {
    uint32_t code[kView][kView];
#pragma unroll
    for (int j = kView - 1; j >= 0; --j) {
      const uint8_t* p = center + (6 - j) * F - 3 * R;
#pragma unroll
      for (int i = 0; i < kView; ++i) {
        code[j][i] = p[0];
        p += R;
      }
    }
#pragma unroll
    for (int j = kView - 1; j >= 0; --j)
#pragma unroll
      for (int i = 0; i < kView; ++i) c[j][i] = table_at(table + kKinds * i, code[j][i]);
  }
};

__device__ __forceinline__ LdsRows lds_rows(const uint32_t* table, const uint8_t* codes, int S, int x,
                                            int y, int dir) {
  // heading 0: ahead +1, right +S; 1: ahead +S, right -1; 2: -1, -S; 3: -S, +1
  const int F = (dir & 1) ? ((dir == 1) ? S : -S) : ((dir == 0) ? 1 : -1);
  const int R = (dir & 1) ? ((dir == 1) ? -1 : 1) : ((dir == 0) ? S : -S);
  return LdsRows{table, codes + y * S + x, R, F};
}

// View rows from the LDS codes with every cell bounds-checked, cells outside
// the grid read as walls: for the rare step whose view can leave the grid,
// through a door on the outer ring that the step itself opened (GoToDoor
// rooms use the grid's border as walls).  The views of such a step are
// computed a second time with these rows.
struct LdsCheckedRows {
  const uint32_t* table;
  const uint8_t* g;   // the env's codes
  int S, x, y, dir;
  __device__ __forceinline__ void load_all(uint32_t (&c)[kView][kView]) const {
    const int fx = dir_dx(dir), fy = dir_dy(dir), rx = -fy, ry = fx;
#pragma unroll
    for (int j = kView - 1; j >= 0; --j)
#pragma unroll
      for (int i = 0; i < kView; ++i) {
        const int wx = x + (i - 3) * rx + (6 - j) * fx, wy = y + (i - 3) * ry + (6 - j) * fy;
        const bool in = (unsigned)wx < (unsigned)S && (unsigned)wy < (unsigned)S;
        c[j][i] = in ? table_at(table + kKinds * i, g[in ? wy * S + wx : 0]) : kCellWall;
      }
  }
};

struct LdsGrid {
  uint8_t* g;
  int S;
  // the 8 cells around interior cell (x, y), row-major, as bits: set = empty
  __device__ __forceinline__ uint32_t free8(int x, int y) const {
    const uint8_t* p = g + (y - 1) * S + (x - 1);
    const uint8_t* q = p + S;
    const uint8_t* r = q + S;
    return (p[0] == 0 ? 1u : 0u) | (p[1] == 0 ? 2u : 0u) | (p[2] == 0 ? 4u : 0u) | (q[0] == 0 ? 8u : 0u) |
           (q[2] == 0 ? 16u : 0u) | (r[0] == 0 ? 32u : 0u) | (r[1] == 0 ? 64u : 0u) | (r[2] == 0 ? 128u : 0u);
  }
  __device__ __forceinline__ void put_empty(int x, int y) const { g[y * S + x] = 0; }
  __device__ __forceinline__ void put_ball(int x, int y) const { g[y * S + x] = (uint8_t)(4u * (19u + kBlue)); }
};

// Whole-grid records straight from the tile's LDS codes (the fused kernel).
// The agents are drawn into the codes beforehand (kinds 51-54, one per
// heading) and removed afterwards, so every output byte is a function of
// the codes alone and needs no staging: the lanes walk the tile's record
// block [0, n) in aligned units held in registers and store each once.
// Symbolic: 16-byte units, at most 6 cells each (18 triple bytes, taken
// from offset r < 3); categorical: 4-byte units of 4 cells, so that
// neighbouring lanes read neighbouring code words.  The units start on the
// 64-byte boundary at or below the block, so that every store instruction
// covers whole 64-byte units of HBM (which writes a partial one as a
// read-modify-write).  Units at the block's two ends store only their bytes
// inside [0, n) (the rest belong to the neighbouring tiles' records); their
// reads reach at most 64 cells before the tile (21 for symbolic units) and
// 7 after it, inside the cleared margins.
// kNT: non-temporal stores (trajectory records); the state write-back
// (emit_dirty_grids) uses ordinary ones, since the next launch reads it again.
// The output bytes of a categorical unit q (4 cells) or a symbolic one (16
// bytes of at most 6 cells), from the LDS codes.
__device__ __forceinline__ uint32_t cat_unit(int o, const uint32_t* table, const uint8_t* codes) {
  // the unit's 4 codes: one aligned word, or two and a byte shift
  const int lo = o & ~3, sh = o & 3;
  const uint32_t* cw = reinterpret_cast<const uint32_t*>(codes + lo);
  const uint32_t c4 = __builtin_amdgcn_alignbyte(cw[1], cw[0], (uint32_t)sh);
  uint32_t ty[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) ty[k] = table_at(table, (c4 >> (8 * k)) & 0xFFu);
  // bytes 0 of the four entries
  return __builtin_amdgcn_perm(__builtin_amdgcn_perm(ty[3], ty[2], 0x0c0c0400u),
                               __builtin_amdgcn_perm(ty[1], ty[0], 0x0c0c0400u), 0x05040100u);
}

__device__ __forceinline__ u32x4 sym_unit(int o, const uint32_t* table, const uint8_t* codes) {
  const int c = (o + 66) / 3 - 22;   // floor(o / 3) for o >= -66
  const uint32_t r = (uint32_t)(o - 3 * c);
  uint32_t t[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) t[k] = table_at(table, codes[c + k]) & 0xFFFFFFu;
  // the 18 bytes t0..t5 as words, then bytes r..r+15 of them
  const uint32_t s0 = t[0] | (t[1] << 24), s1 = (t[1] >> 8) | (t[2] << 16),
                 s2 = (t[2] >> 16) | (t[3] << 8), s3 = t[4] | (t[5] << 24), s4 = t[5] >> 8;
  u32x4 w;
  w.x = __builtin_amdgcn_alignbyte(s1, s0, r);
  w.y = __builtin_amdgcn_alignbyte(s2, s1, r);
  w.z = __builtin_amdgcn_alignbyte(s3, s2, r);
  w.w = __builtin_amdgcn_alignbyte(s4, s3, r);
  return w;
}

template <bool kCat, bool kNT>
__device__ __forceinline__ void store_unit(uintptr_t a, uintptr_t d0, uintptr_t d1, u32x4 w) {
  constexpr int kUnit = kCat ? 4 : 16;
  if (a >= d0 && a + kUnit <= d1) {
    if (kCat) {
      if (kNT) __builtin_nontemporal_store(w.x, reinterpret_cast<uint32_t*>(a));
      else *reinterpret_cast<uint32_t*>(a) = w.x;
    } else {
      if (kNT) __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(a));
      else *reinterpret_cast<u32x4*>(a) = w;
    }
  } else {
#pragma unroll
    for (int b = 0; b < kUnit; ++b)
      if (a + b >= d0 && a + b < d1) reinterpret_cast<uint8_t*>(a)[b] = (uint8_t)(w[b >> 2] >> (8 * (b & 3)));
  }
}

template <bool kCat, bool kNT = true>
__device__ __forceinline__ void emit_tile_grids(uint8_t* dst, int n_cells, const uint32_t* table,
                                                const uint8_t* codes, int lane) {
  constexpr int kUnit = kCat ? 4 : 16;
  // units per lane in flight: all their LDS reads are issued before the
  // first of their stores, so the reads' latency overlaps
  constexpr int kDepth = 4;
  const int64_t n = kCat ? n_cells : 3 * (int64_t)n_cells;
  const uintptr_t d0 = reinterpret_cast<uintptr_t>(dst), d1 = d0 + (uintptr_t)n;
  const uintptr_t A = d0 & ~(uintptr_t)63;
  const int rel = (int)((int64_t)A - (int64_t)d0);   // in [-63, 0]
  const int units = (int)((d1 - A + kUnit - 1) / kUnit);
  for (int q0 = lane; q0 < units; q0 += kDepth * kWave) {
    // a unit past the block's last one reads that last unit's cells again
    u32x4 w[kDepth];
#pragma unroll
    for (int u = 0; u < kDepth; ++u) {
      const int o = rel + kUnit * min(q0 + u * kWave, units - 1);   // output byte of the unit's first byte
      if (kCat) w[u] = u32x4{cat_unit(o, table, codes), 0u, 0u, 0u};
      else w[u] = sym_unit(o, table, codes);
    }
#pragma unroll
    for (int u = 0; u < kDepth; ++u) {
      const int q = q0 + u * kWave;
      if (q < units) store_unit<kCat, kNT>(A + (uintptr_t)(kUnit * q), d0, d1, w[u]);
    }
  }
}

// Write-back of the grids that changed in a launch (the lanes with `dirty`
// set; every other env's grid in HBM still holds the bytes staged in, so
// writing it again would change nothing).  The dirty lanes mark the 64-byte
// lines of the tile's block that their grids touch, in a bitmap in `lines`
// (LDS, one bit per line), and the symbolic units of emit_tile_grids are
// then stored for the marked lines only: a line's other bytes belong to
// neighbouring envs and are rewritten with their current cells, which equal
// what HBM holds, and the units at the block's two ends store only their
// bytes inside it.
__device__ __forceinline__ void emit_dirty_grids(uint8_t* dst, int n_cells, bool dirty, int my_off, int my_cells,
                                                 const uint32_t* table, const uint8_t* codes, uint32_t* lines,
                                                 int lane) {
  const uintptr_t d0 = reinterpret_cast<uintptr_t>(dst), d1 = d0 + 3 * (uintptr_t)(uint32_t)n_cells;
  const uintptr_t A = d0 & ~(uintptr_t)63;
  const int rel = (int)((int64_t)A - (int64_t)d0);   // in [-63, 0]
  const int units = (int)((d1 - A + 15) / 16);
  const int n_words = (((units + 3) >> 2) + 31) >> 5;
  for (int w = lane; w < n_words; w += kWave) lines[w] = 0u;
  wave_sync();
  if (dirty && my_cells > 0) {
    // lines [l0, l1) hold this grid's bytes; at most 49 lines, so 3 words
    const int l0 = (3 * my_off - rel) >> 6, l1 = (3 * (my_off + my_cells) - rel + 63) >> 6;
    for (int w = l0 >> 5; w <= (l1 - 1) >> 5; ++w) {
      const int lo = max(l0 - 32 * w, 0), hi = min(l1 - 32 * w, 32);
      atomicOr(&lines[w], (hi - lo == 32 ? ~0u : ((1u << (hi - lo)) - 1u)) << lo);
    }
  }
  wave_sync();
  constexpr int kDepth = 4;
  for (int qb = lane; qb < units; qb += kDepth * kWave) {
    u32x4 w[kDepth];
    bool keep[kDepth];
#pragma unroll
    for (int u = 0; u < kDepth; ++u) {
      const int q = qb + u * kWave;
      keep[u] = q < units && ((lines[q >> 7] >> ((q >> 2) & 31)) & 1u) != 0;
      w[u] = keep[u] ? sym_unit(rel + 16 * q, table, codes) : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int u = 0; u < kDepth; ++u)
      if (keep[u]) store_unit<false, false>(A + (uintptr_t)(16 * (qb + u * kWave)), d0, d1, w[u]);
  }
}

// Kind codes of triples by table: entry type << 5 | colour << 2 | state
// (types 0-15, colours 0-7, states 0-3) holds code_of of that triple.  A
// valid grid holds only types 0-9, colours 0-5 and states 0-2, so its every
// cell gets code_of's code for five instructions and one LDS read instead
// of code_of's fifteen; bits of a triple beyond those fields are ignored.
// The table lives in the record stage while a tile is staged in.
constexpr int kCodeLutBytes = 512;

__device__ __forceinline__ void build_code_lut(uint8_t* lut, int lane) {
#pragma unroll
  for (int k = 0; k < kCodeLutBytes / kWave; ++k) {
    const uint32_t i = (uint32_t)(lane + k * kWave);
    lut[i] = (uint8_t)code_of((i >> 5) | (((i >> 2) & 7u) << 8) | ((i & 3u) << 16));
  }
}

__device__ __forceinline__ uint32_t lut_code(const uint8_t* lut, uint32_t tri) {
  const uint32_t i = ((tri & 15u) << 5) | (((tri >> 8) & 7u) << 2) | ((tri >> 16) & 3u);
  return lut[i];
}

// Stages a tile's grids, the 3 * n_cells bytes at src (any alignment), into
// LDS as codes.  Lane u converts cells [16u, 16u + 16), i.e. the 48 bytes
// at src + 48u; 48 being a multiple of 16, every such run starts at the
// same offset r = src mod 16 in its first aligned 16-byte chunk, so a run is
// four aligned chunk loads and one realignment by the wave-uniform r (the
// conversion is instantiated per r / 4, so the realignment needs no
// selects).  A chunk past the block's last one is read as that last chunk
// (so every load lies in the block's own memory pages); the codes of the at
// most 15 cells past n_cells land in the trailing LDS margin, which needs
// nothing but valid codes, and every table entry is one.  The lane's next
// run is loaded before its current run is converted, so the wave's reads
// stay in flight while it converts.
struct GridRun {
  u32x4 q[4];
};

__device__ __forceinline__ GridRun load_run(uintptr_t a, uintptr_t last) {
  GridRun g;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uintptr_t c = a + 16 * (uintptr_t)k;
    g.q[k] = *reinterpret_cast<const u32x4*>(c < last ? c : last);
  }
  return g;
}

template <int kRW>
__device__ __forceinline__ void convert_run(const GridRun& g, uint32_t rb, const uint8_t* lut, uint8_t* dst) {
  uint32_t w[16];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) w[4 * k + c] = g.q[k][c];
  // bytes r .. r + 47 of the chunks as 12 words (r = 4 kRW + rb)
  uint32_t b[12];
#pragma unroll
  for (int i = 0; i < 12; ++i)
    b[i] = i + kRW + 1 < 16 ? __builtin_amdgcn_alignbyte(w[i + kRW + 1], w[i + kRW], rb) : w[i + kRW] >> (8 * rb);
  uint32_t out[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int d = (3 * k) >> 2, off = (3 * k) & 3;
    const uint32_t tri = d + 1 < 12 ? __builtin_amdgcn_alignbyte(b[d + 1], b[d], (uint32_t)off)
                                    : b[d] >> (8 * off);
    out[k >> 2] |= lut_code(lut, tri) << (8 * (k & 3));
  }
  *reinterpret_cast<u32x4*>(dst) = u32x4{out[0], out[1], out[2], out[3]};
}

template <int kRW>
__device__ __forceinline__ void stage_in_runs(uintptr_t a0, uintptr_t last, uint32_t rb, int units,
                                              const uint8_t* lut, uint8_t* codes, int lane) {
  int u = lane;
  if (u >= units) return;
  GridRun cur = load_run(a0 + 48 * (uintptr_t)u, last);
  while (true) {
    const int nu = u + kWave;
    const bool more = nu < units;
    GridRun nxt;
    if (more) nxt = load_run(a0 + 48 * (uintptr_t)nu, last);
    convert_run<kRW>(cur, rb, lut, codes + 16 * u);
    if (!more) break;
    cur = nxt;
    u = nu;
  }
}

// lut: the code table (build_code_lut), visible to every lane
__device__ __forceinline__ void stage_in_codes(const uint8_t* src, int n_cells, uint8_t* codes,
                                               const uint8_t* lut, int lane) {
  const uintptr_t s0 = reinterpret_cast<uintptr_t>(src);
  const uint32_t r = (uint32_t)__builtin_amdgcn_readfirstlane((int)(s0 & 15u));
  const uintptr_t end = s0 + 3 * (uintptr_t)(uint32_t)n_cells;
  const uintptr_t a0 = s0 - r, last = (end - 1) & ~(uintptr_t)15;
  const int units = (n_cells + 15) >> 4;
  switch (r >> 2) {
    case 0: stage_in_runs<0>(a0, last, r & 3u, units, lut, codes, lane); break;
    case 1: stage_in_runs<1>(a0, last, r & 3u, units, lut, codes, lane); break;
    case 2: stage_in_runs<2>(a0, last, r & 3u, units, lut, codes, lane); break;
    default: stage_in_runs<3>(a0, last, r & 3u, units, lut, codes, lane); break;
  }
}

// Writes the code grids of the freshly laid-out envs in `pending` (a lane
// mask; each such lane holds its Layout) into LDS at codes + its offset: the
// whole wave fills one grid at a time, 64 cells per pass in row-major order.
__device__ __forceinline__ void fill_layouts(uint64_t pending, const Layout& L, uint8_t* codes, int my_off,
                                             int lane) {
  while (pending) {
    const int r = __ffsll((unsigned long long)pending) - 1;
    pending &= pending - 1;
    const Layout Lr = bcast_layout(L, r);
    uint8_t* gp = codes + bcast(my_off, r);
    const uint32_t Sr = (uint32_t)Lr.S;
    uint32_t yy, xx, dy, dx;
    small_divmod((uint32_t)lane, Sr, yy, xx);
    small_divmod((uint32_t)kWave, Sr, dy, dx);
    for (uint32_t c = (uint32_t)lane; c < Sr * Sr; c += kWave) {
      gp[c] = (uint8_t)layout_code(Lr, (int)xx, (int)yy);
      xx += dx;
      yy += dy;
      const bool wrap = xx >= Sr;
      xx -= wrap ? Sr : 0u;
      yy += wrap ? 1u : 0u;
    }
  }
}

struct FusedArgs {
  EnvTables env;
  TileTables tiles;
  StateBufs st;
  const uint8_t* actions;   // [k_steps][N] or nullptr
  int32_t k_steps;
  TrajBufs out;
  int32_t row0;
  ServeTile* serve;               // per-tile requests (serving), else nullptr
  const ServeTile* host_tiles;    // serving: staging of newly admitted tiles (pinned host memory)
  const SlotConfig* host_slots;   // serving: their slot configurations
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

// kActions: actions come from a.actions; otherwise from the random policy.
// kServe: tiles belong to requests described by a.serve (serving): each runs
// min(K, steps it has left) steps from its own counter step0, writes to its
// own output rows and advances step0.
// kObs: the observation records written, 0 symbolic first person, 1
// categorical first person, 2 whole grid (a.env.obs_mode 2 or 3); each
// variant carries only its own record code.
// On this GPU one counter tracks both outstanding loads and stores, so a
// load consumed in the same step would also wait for every earlier record
// store: the action of step s + 1 is therefore fetched during step s, and
// the policy variant has no loads in its step loop at all.
template <bool kActions, bool kServe, int kObs>
__global__ __launch_bounds__(kWave) void k_fused(FusedArgs a) {
  // static LDS (table and record stage) sits at fixed addresses, so table
  // reads take their base as an immediate; the tile grids are dynamic
  __shared__ __align__(16) uint32_t table[kKinds * kView];
  __shared__ __align__(16) uint8_t stage[kRecStageBytes];
  // per lane: whether a pickup, drop or toggle changed a cell of its grid
  __shared__ uint8_t cell_changed[kWave];
  extern __shared__ __align__(16) uint8_t grids[];
  uint8_t* codes = grids + kMargin;
  const int lane = threadIdx.x;
  const int N = a.env.n;

  {
    const uint32_t t = triple_of_kind((uint32_t)lane);   // kKinds == kWave entries
#pragma unroll
    for (int i = 0; i < kView; ++i) table[kKinds * i + lane] = (t & ~kSeeBit) | ((t & kSeeBit) >> i);
  }
  // Every byte a view may read holds a code from here on: the margins and
  // any space past a small tile are cleared once (code 0, an empty cell),
  // and the kernel only ever writes codes.  An arbitrary byte would index
  // the tables off an entry boundary and could set another column's
  // see-through flag, which the row's combined flags would then pick up.
  {
    const uint32_t quads = (uint32_t)(tile_lds_bytes(a.tiles.max_tile_cells) >> 4);
    for (uint32_t w = (uint32_t)lane; w < quads; w += kWave)
      reinterpret_cast<u32x4*>(grids)[w] = u32x4{0u, 0u, 0u, 0u};
  }
  wave_sync();

  for (int it = blockIdx.x; it < a.tiles.n_tiles; it += gridDim.x) {
    // serving lists mark a newly admitted tile with the top bit: its
    // descriptor and slot configurations are still in host staging and its
    // envs are reset here (episode 0) before its first step
    const uint32_t entry = a.tiles.list ? a.tiles.list[it] : (uint32_t)it;
    const int tile = (int)(entry & 0x7FFFFFFFu);
    const bool fresh = kServe && (entry >> 31) != 0;
    // where this tile's envs live and where their records go: record of
    // step s, lane l is at index rec_base + s * rec_step (+ l) of the outputs
    const int tile_envs = kServe ? kWave : a.tiles.tile_envs;
    const int e0 = tile * tile_envs;
    int n_here, steps;
    uint64_t g0 = 0;
    uint8_t *o_obs, *o_flags, *o_action, *o_mission = nullptr;
    float* o_reward;
    uint32_t step0 = 0;
    size_t rec_stride;
    if (kServe) {
      const ServeTile d = fresh ? a.host_tiles[tile] : a.serve[tile];
      if (fresh && lane == 0) a.serve[tile] = d;   // the device copy later launches read
      if (!d.active || d.step0 >= d.n_steps) continue;
      n_here = (int)d.n_envs;
      steps = min(a.k_steps, (int)(d.n_steps - d.step0));
      step0 = d.step0;
      g0 = d.grid_base;
      o_obs = d.obs;
      o_reward = d.reward;
      o_flags = d.flags;
      o_action = d.action;
      rec_stride = d.stride;
      o_obs = o_obs ? o_obs + (size_t)d.local0 * kObsBytes : nullptr;
      o_reward += d.local0;
      o_flags += d.local0;
      o_action += d.local0;
    } else {
      n_here = min(tile_envs, N - e0);
      steps = a.k_steps;
      o_obs = a.out.obs ? a.out.obs + (size_t)e0 * (kObs == 1 ? kCatBytes : kObsBytes) : nullptr;
      o_reward = a.out.reward + e0;
      o_flags = a.out.flags + e0;
      o_action = a.out.action + e0;
      o_mission = a.out.mission ? a.out.mission + e0 : nullptr;
      rec_stride = (size_t)N;
    }
    const int e = e0 + lane;
    const bool active = lane < n_here;

    uint32_t fam = 0, meta = 0;
    int S = 0, T = 1, x = 1, y = 1, dir = 0, t = 0;
    uint32_t carry = kCellEmpty, episode = 0, rid = 0, calls = 0;
    bool done_prev = false;
    uint2 seed = make_uint2(0, 0);
    uint64_t goff = 0;
    uint32_t ob[4] = {~0u, ~0u, ~0u, ~0u};
    Layout L0{};
    if (active && fresh) {
      const SlotConfig c = a.host_slots[e];
      meta = c.meta;
      T = c.max_steps;
      seed = c.seed;
      rid = c.rng_id;
      a.env.meta[e] = c.meta;
      a.env.max_steps[e] = c.max_steps;
      a.env.seed[e] = c.seed;
      a.env.rng_id[e] = c.rng_id;
      a.env.grid_off[e] = c.grid_off;
      fam = meta & 0xFF;
      S = (int)((meta >> 8) & 0xFF);
      L0 = make_layout(meta, seed, rid, 0u);
      x = L0.ax;
      y = L0.ay;
      dir = L0.dir;
#pragma unroll
      for (int i = 0; i < 4; ++i) ob[i] = L0.ob[i];
    } else if (active) {
      meta = a.env.meta[e];
      fam = meta & 0xFF;
      S = (int)((meta >> 8) & 0xFF);
      T = a.env.max_steps[e];
      seed = a.env.seed[e];
      rid = a.env.rng_id[e];
      if (!kServe) goff = a.env.grid_off[e];
      x = a.st.x[e];
      y = a.st.y[e];
      dir = a.st.dir[e];
      t = a.st.t[e];
      carry = (uint32_t)a.st.carry[e];
      episode = a.st.episode[e];
      done_prev = a.st.done_prev[e] != 0;
      calls = a.st.calls[e];
      const uint4 o4 = *reinterpret_cast<const uint4*>(a.st.obst + 16 * (size_t)e);
      ob[0] = o4.x; ob[1] = o4.y; ob[2] = o4.z; ob[3] = o4.w;
    }
    int tile_cells;
    const int my_off = wave_excl_scan(S * S, lane, tile_cells);
    cell_changed[lane] = 0;
    uint8_t* my_codes = codes + my_off;
    // the tile's grids are contiguous in HBM: stage them as codes (a fresh
    // tile's are laid out here instead)
    if (!kServe) g0 = (uint64_t)__shfl((long long)goff, 0, kWave);
    if (fresh) {
      fill_layouts(__ballot(active), L0, codes, my_off, lane);
    } else {
      // the record stage is idle until the first step: it holds the code table
      build_code_lut(stage, lane);
      wave_sync();
      stage_in_codes(a.st.grid + g0, tile_cells, codes, stage, lane);
    }
    wave_sync();

    uint4 pol = make_uint4(0, 0, 0, 0);
    uint32_t act_next = 0;
    if (kActions && active) act_next = a.actions[e];
    for (int s = 0; s < steps; ++s) {
      // the env's call count; envs stepped together share it, so the policy
      // block refresh every 4 calls is uniform across the wave in practice
      const uint32_t call = calls + (uint32_t)s;
      uint32_t act_now = 0;
      if (kActions) {
        act_now = act_next;
        if (active && s + 1 < steps) act_next = a.actions[(size_t)(s + 1) * N + e];
      } else if (s == 0 || (call & 3) == 0) {
        pol = policy_block(seed, rid, call);
      }

      const bool do_reset = active && done_prev;
      Layout L{};
      if (do_reset) {
        episode += 1u;
        L = make_layout(meta, seed, rid, episode);
        x = L.ax;
        y = L.ay;
        dir = L.dir;
        t = 0;
        carry = kCellEmpty;
#pragma unroll
        for (int i = 0; i < 4; ++i) ob[i] = L.ob[i];
      }
      const uint64_t pending = __ballot(do_reset);
      if (pending) {
        fill_layouts(pending, L, codes, my_off, lane);
        wave_sync();
      }

      float reward = 0.0f;
      uint32_t flags = 0, act_rec = kActionNone;
      bool edge_view = false;
      if (active && !do_reset) {
        uint32_t act = kActions ? act_now : bounded(pick4(pol, call & 3u), 7u);
        const int fx = x + dir_dx(dir), fy = y + dir_dy(dir);
        uint32_t front = table_at(table, my_codes[fy * S + fx]);
        bool blocked = false;
        if (fam == kFamDynObs) {
          // three actions; the cell ahead is judged before the balls move
          act = act > kForward ? kLeft : act;
          blocked = (front & 0xFF) != kEmpty && (front & 0xFF) != kGoal;
          move_obstacles(LdsGrid{my_codes, S}, (int)((meta >> 16) & 0xFF), x, y, ob, seed, rid, call);
          front = table_at(table, my_codes[fy * S + fx]);
        }
        ActResult r = intervene(act, x, y, dir, carry, front, fx, fy);
        r.penalty = r.penalty || (blocked && act == kForward);
        r.terminated = r.terminated || r.penalty;
        if (fam == kFamGoToDoor) {
          gotodoor_rules(r, act, front, ob[0] & 0xFFu);
          edge_view = r.front_changed;   // a door toggled, possibly on the outer ring
        }
        if (r.front_changed) {
          my_codes[fy * S + fx] = (uint8_t)code_of(r.new_front);
          cell_changed[lane] = 1;
        }
        t += 1;
        const bool trunc = t >= T;
        reward = step_reward(r, t, T, a.env.reward_mode);
        flags = (r.terminated ? kFlagTerminated : 0u) | (trunc ? kFlagTruncated : 0u);
        done_prev = r.terminated || trunc;
        act_rec = act & 0xFF;
      } else if (do_reset) {
        flags = kFlagFirst;
        done_prev = false;
      }

      const size_t row = kServe ? (size_t)(step0 + s) : (size_t)((a.row0 + s) % a.out.rows);
      const size_t rec = row * rec_stride;   // index of lane 0's record
      if (kObs == 2 && o_obs && !kServe) {
        // whole-grid records, packed like the tile's grids (from g0): the
        // agents are drawn into the codes for the copy and then removed
        uint8_t* at = my_codes + y * S + x;
        uint8_t under = 0;
        if (active) {
          under = *at;
          *at = (uint8_t)(4u * (kAgentKind + (uint32_t)dir));
        }
        wave_sync();   // every lane's grid writes of this step, and the agents
        uint8_t* dst = a.out.obs + row * a.out.obs_row;
        if (a.env.obs_mode == 3) emit_tile_grids<true>(dst + g0 / 3, tile_cells, table, codes, lane);
        else emit_tile_grids<false>(dst + g0, tile_cells, table, codes, lane);
        wave_sync();
        if (active) *at = under;
      } else if (kObs == 1 && o_obs && !kServe) {
        // categorical records (49 bytes): the stage holds all 64 at once
        uint32_t u[kObsWords + 1];
        observe_words<true>(lds_rows(table, my_codes, S, x, y, dir), carry, active, lane, u);
        if (__ballot(edge_view))
          observe_words<true>(LdsCheckedRows{table, my_codes, S, x, y, dir}, carry, active, lane, u);
        store_words<true>(stage, lane, u);
        wave_sync();
        copy_out<kWave, kCatBytes>(stage, o_obs + rec * kCatBytes, n_here, lane);
        wave_sync();
      } else if (kObs == 0 && o_obs) {
        // inactive lanes (S = 0, pose (1, 1)) read inside the guard margin
        uint32_t u[kObsWords + 1];
        observe_words<false>(lds_rows(table, my_codes, S, x, y, dir), carry, active, lane & 31, u);
        if (__ballot(edge_view))
          observe_words<false>(LdsCheckedRows{table, my_codes, S, x, y, dir}, carry, active, lane & 31, u);
        // the stage holds 32 records: lanes 0-31, then lanes 32-63 (each half
        // starts and ends on a word boundary, so the halves are independent).
        // HBM writes whole 64-byte units: a store that covers only part of
        // one costs a read-modify-write, and so does a unit that two pieces
        // of the block share, since they leave at different times.  So the
        // first piece ends on a 64-byte boundary of the output and its last
        // `keep` bytes (< 64) are moved to the front of the stage, with the
        // second half staged right behind them.
        uint8_t* dst = o_obs + rec * kObsBytes;
        const int n_first = min(32, n_here);
        const int bytes0 = n_first * kObsBytes;
        const uintptr_t d = reinterpret_cast<uintptr_t>(dst);
        const int keep = (n_here > 32 && (d & 15) == 0) ? (int)((d + (uintptr_t)bytes0) & 63) : 0;
        if (lane < 32) store_words<false>(stage, lane, u);
        wave_sync();
        copy_piece<kHalfStageBytes>(stage, dst, bytes0 - keep, lane);
        if (n_here > 32) {
          // source [bytes0 - keep, bytes0) and destination [0, keep) are disjoint
          if (lane < (keep >> 4)) {
            const u32x4 v = *reinterpret_cast<const u32x4*>(stage + bytes0 - keep + 16 * lane);
            *reinterpret_cast<u32x4*>(stage + 16 * lane) = v;
          }
          wave_sync();
          if (lane >= 32) store_words<false>(stage + keep, lane & 31, u);
          wave_sync();
          copy_piece<kRecStageBytes>(stage, dst + bytes0 - keep, keep + (n_here - 32) * kObsBytes, lane);
        }
        wave_sync();
      }
      if (active) {
        o_reward[rec + lane] = reward;
        o_flags[rec + lane] = (uint8_t)flags;
        o_action[rec + lane] = (uint8_t)act_rec;
        if (o_mission) o_mission[rec + lane] = (uint8_t)mission_of(fam, ob[0]);
      }
      wave_sync();
    }

    // write the chunk's final state back: the grids that changed (laid out
    // afresh, by a reset (the episode counter moved on from the one still
    // in HBM) or at admission, written by a pickup, drop or toggle, or
    // holding balls, which move every step)
    const bool dirty = active && (fresh || fam == kFamDynObs || cell_changed[lane] != 0 ||
                                  episode != a.st.episode[e]);
    // the record stage is idle after the last step: it holds the line bitmap
    // (a tile of 64 grids of side 32 spans at most 3074 lines)
    static_assert(((3 * kWave * 32 * 32 + 63 + 15) / 16 / 4 + 1 + 31) / 32 * 4 <= kRecStageBytes,
                  "the line bitmap fits the record stage");
    emit_dirty_grids(a.st.grid + g0, tile_cells, dirty, my_off, S * S, table, codes,
                     reinterpret_cast<uint32_t*>(stage), lane);
    if (active) {
      a.st.x[e] = x;
      a.st.y[e] = y;
      a.st.dir[e] = dir;
      a.st.t[e] = t;
      a.st.carry[e] = (int32_t)carry;
      a.st.episode[e] = episode;
      a.st.done_prev[e] = done_prev ? 1 : 0;
      a.st.calls[e] = calls + (uint32_t)steps;
      *reinterpret_cast<uint4*>(a.st.obst + 16 * (size_t)e) = make_uint4(ob[0], ob[1], ob[2], ob[3]);
    }
    if (kServe && lane == 0) a.serve[tile].step0 = step0 + (uint32_t)steps;
    wave_sync();
  }
}

}  // namespace

size_t fused_dynamic_lds_bytes(int32_t max_tile_cells) { return tile_lds_bytes(max_tile_cells); }

size_t fused_lds_bytes(int32_t max_tile_cells) {
  return kKinds * kView * 4 + kRecStageBytes + kWave + fused_dynamic_lds_bytes(max_tile_cells);
}

hipError_t launch_plain(const EnvTables& env, const StateBufs& st, const uint8_t* actions,
                        int reset_all, const TrajBufs& out, int32_t row, hipStream_t stream) {
  PlainArgs a{env, st, actions, reset_all, out, row};
  const int blocks = (env.n + kWave - 1) / kWave;
  hipLaunchKernelGGL(k_plain, dim3(blocks), dim3(kWave), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_fused(const EnvTables& env, const TileTables& tiles, const StateBufs& st,
                        const uint8_t* actions, int32_t k_steps,
                        const TrajBufs& out, int32_t row0, int32_t grid_blocks,
                        hipStream_t stream, ServeTile* serve, const ServeTile* host_tiles,
                        const SlotConfig* host_slots) {
  FusedArgs a{env, tiles, st, actions, k_steps, out, row0, serve, host_tiles, host_slots};
  const size_t lds = fused_dynamic_lds_bytes(tiles.max_tile_cells);
  // serving requests record symbolic first-person observations
  const int obs = serve ? 0 : (env.obs_mode >= 2 ? 2 : env.obs_mode);
  using Kernel = void (*)(FusedArgs);
  static const Kernel kernels[2][3] = {
      {&k_fused<false, false, 0>, &k_fused<false, false, 1>, &k_fused<false, false, 2>},
      {&k_fused<true, false, 0>, &k_fused<true, false, 1>, &k_fused<true, false, 2>}};
  const Kernel fn = serve ? &k_fused<false, true, 0> : kernels[actions ? 1 : 0][obs];
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(grid_blocks), dim3(kWave), lds, stream, a);
  return hipGetLastError();
}

}  // namespace gx
