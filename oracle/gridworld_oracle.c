/*
 * gridworld_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU model of the batched gridworld
 * environment step of NAVIX (Pignatelli et al., "NAVIX: Scaling MiniGrid
 * Environments with JAX", arXiv 2407.19396).  It exists to check the HIP
 * path; nothing in the product may link, import or execute it.  Only the
 * tests, the smoke entry and the CPU-baseline leg of the benchmark use it.
 *
 * It shares no code, header, table or constant with the GPU library.
 *
 * What it follows:
 *   - the timestep protocol and autoreset (Sec. 3.2.2: the timestep tuple,
 *     the reset padding the action with -1 and the reward with 0, and a
 *     step that resets by itself once the episode has ended);
 *   - the systems in their order: intervention, transition, observation,
 *     reward, termination (Table "systems"; App. A);
 *   - the entities and components (Tables "components", "entities"):
 *     walls, doors (openable, possibly locked), keys (pickable), goal;
 *   - the reward of Sec. 3.2.1 / Eq. (1) in the time-discounted form
 *     r = 1 - 0.9 * (t / T) evaluated in IEEE fp32, with t the number of
 *     steps since reset after the current one, or the Markovian unit reward
 *     the paper defaults to (reward_mode 1);
 *   - the first-person symbolic observation (Table "observations",
 *     symbolic_first_person, R = 7) with MiniGrid's occlusion rule, since
 *     Sec. 3.2.1 states the environments match MiniGrid exactly, and the
 *     other observation functions of that table: categorical_first_person,
 *     symbolic and categorical, and the images rgb_first_person and rgb,
 *     drawn from a sprite atlas the caller passes in;
 *   - the Empty, DoorKey (two rooms) and FourRooms families (Table "envs"),
 *     and the lava families LavaGap, Crossings and DistShift with the
 *     goal-or-lava reward R2 of Table "envs" (lava: -1 and termination,
 *     Tables "rewards" and "terminations", on_lava_fall);
 *   - Dynamic-Obstacles (Table "envs", reward R3; Fig. 1): balls that move
 *     at random every step, the first family whose transition system is
 *     not the identity (Table "systems");
 *   - GoToDoor (on_door_done of Tables "rewards" and "terminations"; its
 *     mission is part of the state) and KeyCorridor (reward R1), the last
 *     families of Table "envs".
 *
 * Every point the paper leaves open is fixed by a documented reading; the
 * readings are listed next to each function.  Parity status of each
 * function is stated in its comment ("pinned by" / "parity unpinned").
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * No FMA contraction: the reward must be three separately rounded fp32
 * operations.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- encoding (MiniGrid's canonical object/colour/state indices) ---- */
enum { O_UNSEEN = 0, O_EMPTY = 1, O_WALL = 2, O_FLOOR = 3, O_DOOR = 4,
       O_KEY = 5, O_BALL = 6, O_BOX = 7, O_GOAL = 8, O_LAVA = 9,
       O_AGENT = 10 };
enum { C_RED = 0, C_GREEN = 1, C_BLUE = 2, C_PURPLE = 3, C_YELLOW = 4,
       C_GREY = 5 };
enum { D_OPEN = 0, D_CLOSED = 1, D_LOCKED = 2 };
/* actions (MiniGrid order): left, right, forward, pickup, drop, toggle, done */
enum { A_LEFT = 0, A_RIGHT = 1, A_FORWARD = 2, A_PICKUP = 3, A_DROP = 4,
       A_TOGGLE = 5, A_DONE = 6 };
enum { FAM_EMPTY = 0, FAM_TWOROOM = 1, FAM_FOURROOMS = 2, FAM_LAVAGAP = 3,
       FAM_CROSSINGS = 4, FAM_DISTSHIFT = 5, FAM_DYNOBS = 6, FAM_GOTODOOR = 7,
       FAM_KEYCORRIDOR = 8 };
#define OX_MAX_OBST 8

#define OX_FLAG_TERMINATED 1u
#define OX_FLAG_TRUNCATED 2u
#define OX_FLAG_FIRST 4u
#define OX_ACTION_NONE 0xFFu
#define OX_VIEW 7

/* direction d: 0 = +x (east), 1 = +y (south), 2 = -x (west), 3 = -y (north) */
static const int DIR_X[4] = {1, 0, -1, 0};
static const int DIR_Y[4] = {0, 1, 0, -1};

/* ------------------------------------------------------------------ */
/* Philox4x32-10, written from Salmon, Moraes, Dror, Shaw, "Parallel   */
/* random numbers: as easy as 1, 2, 3" (SC'11), Sec. 3.3 / Table 2:    */
/* each round multiplies counter words 0 and 2 by the two round         */
/* multipliers, swaps in the high halves xored with the other words and */
/* the round key, and the key is advanced by the two Weyl constants     */
/* between rounds.  Pinned by the known-answer vectors of that paper's  */
/* reference distribution (tests/golden/philox_kat.json).               */
/* ------------------------------------------------------------------ */
void ox_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                      uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform integer in [0, n): floor(word * n / 2^32). */
uint32_t ox_uniform(uint32_t word, uint32_t n) {
  return (uint32_t)(((uint64_t)word * (uint64_t)n) >> 32);
}

/* Random words of one layout draw: key = seed, counter =
 * (rng_id, episode, word_index / 4, 0); word w is lane w % 4. */
static uint32_t layout_word(uint64_t seed, uint32_t rng_id, uint32_t episode,
                            uint32_t w) {
  uint32_t ctr[4] = {rng_id, episode, w / 4u, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  ox_philox4x32_10(ctr, key, out);
  return out[w % 4u];
}

/* Random-policy action of an env's step call number `call` (its step calls
 * since its reset, the autoresetting ones included): counter = (rng_id,
 * (call / 4) low 32 bits, (call / 4) high 32 bits, 1), lane call % 4,
 * uniform over the 7 actions.  The action drawn on a call that autoresets
 * is not used. */
uint32_t ox_policy_action(uint64_t seed, uint32_t rng_id, uint64_t call) {
  uint64_t block = call / 4u;
  uint32_t ctr[4] = {rng_id, (uint32_t)block, (uint32_t)(block >> 32), 1u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  ox_philox4x32_10(ctr, key, out);
  return ox_uniform(out[call % 4u], 7u);
}

/* ------------------------------------------------------------------ */
/* grid helpers: grid is [y][x][3] bytes (type, colour, state)         */
/* ------------------------------------------------------------------ */
static uint8_t *cell(uint8_t *g, int S, int x, int y) {
  return g + 3 * (y * S + x);
}
static void put(uint8_t *g, int S, int x, int y, int type, int colour,
                int state) {
  uint8_t *c = cell(g, S, x, y);
  c[0] = (uint8_t)type; c[1] = (uint8_t)colour; c[2] = (uint8_t)state;
}

/* The k-th cell (0-based, row-major: y then x) inside the rectangle
 * [x0,x1] x [y0,y1] whose type is empty.  Returns 0 on success. */
static int kth_empty(const uint8_t *g, int S, int x0, int x1, int y0, int y1,
                     uint32_t k, int *ox, int *oy) {
  uint32_t seen = 0;
  for (int y = y0; y <= y1; ++y)
    for (int x = x0; x <= x1; ++x) {
      if (g[3 * (y * S + x)] != O_EMPTY) continue;
      if (seen == k) { *ox = x; *oy = y; return 0; }
      ++seen;
    }
  return -1;
}
static uint32_t count_empty(const uint8_t *g, int S, int x0, int x1, int y0,
                            int y1) {
  uint32_t n = 0;
  for (int y = y0; y <= y1; ++y)
    for (int x = x0; x <= x1; ++x)
      if (g[3 * (y * S + x)] == O_EMPTY) ++n;
  return n;
}

/* Side (and parameter) limits of each family.  The parameter is the
 * number of lava rivers of Crossings (at most 8 and at most S - 3), the
 * variant (1 or 2) of DistShift, the number of obstacles (1 to 8, leaving
 * two free interior cells) of Dynamic-Obstacles and the rows of rooms (1 to
 * 3) of KeyCorridor; the other families ignore it. */
int ox_side_ok(int family, int side, int param) {
  if (side > 32) return 0;
  switch (family) {
    case FAM_EMPTY: return side >= 4;
    case FAM_TWOROOM: return side >= 5;
    case FAM_FOURROOMS: return side >= 7 && (side % 2) == 1;
    case FAM_LAVAGAP: return side >= 5;
    case FAM_CROSSINGS:
      return side >= 5 && (side % 2) == 1 && param >= 1 && param <= 8 && param <= side - 3;
    case FAM_DISTSHIFT: return side >= 6 && (param == 1 || param == 2);
    case FAM_DYNOBS:
      return side >= 5 && param >= 1 && param <= OX_MAX_OBST &&
             param <= (side - 2) * (side - 2) - 2;
    case FAM_GOTODOOR: return side >= 5;
    case FAM_KEYCORRIDOR:   /* side = 3 s - 2 for rooms of size s >= 3; param = rows 1..3 */
      return side >= 7 && (side + 2) % 3 == 0 && param >= 1 && param <= 3;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Start-state distribution P0 (Sec. 3.2.2, reset(key); Table "envs"  */
/* for the families; App. D, custom-env _reset: build the grid, place */
/* the entities).  Draws are taken from the layout stream in the      */
/* order written.  "Uniform placement" = the k-th empty cell of the   */
/* region in row-major order, k uniform over the count.               */
/*                                                                     */
/* Empty(S): wall border, goal (green) at (S-2, S-2); agent uniform    */
/*   over the empty interior; direction uniform.                       */
/* TwoRoom(S) (DoorKey): wall column c = 2 + u(S-4); door row          */
/*   d = 1 + u(S-3); door colour u(6), locked; goal at (S-2, S-2); key */
/*   of the door's colour uniform over the empty cells of the left     */
/*   room x in [1, c-1]; agent uniform over the remaining empty cells  */
/*   of the left room; direction uniform.                              */
/* FourRooms(S odd): walls along row m and column m, m = S / 2; one    */
/*   opening per wall segment, drawn in the order (m, 1+u(m-1)),       */
/*   (m, m+1+u(m-1)), (1+u(m-1), m), (m+1+u(m-1), m); goal uniform     */
/*   over all empty cells, agent uniform over the remaining empty      */
/*   cells; direction uniform.                                          */
/* The lava families start the agent at (1, 1) facing east with the    */
/* goal in a fixed corner, as MiniGrid's versions of them do:          */
/* LavaGap(S): goal (S-2, S-2); lava column c = 2 + u(S-4), full over  */
/*   rows 1..S-2 except the gap row 1 + u(S-2).                         */
/* Crossings(S odd, N rivers): goal (S-2, S-2).  Candidate rivers are  */
/*   the columns x = 2, 4, .., S-3 then the rows y = 2, 4, .., S-3;     */
/*   N of them are chosen by a partial Fisher-Yates shuffle (step k    */
/*   swaps candidate k with candidate k + u(M - k), M = S - 3).  Each   */
/*   chosen river is a full lava line across the interior.  The rivers */
/*   cut the interior into a lattice of rooms; a monotone path of room */
/*   moves from the top-left room to the bottom-right one is drawn one */
/*   move at a time (east with probability rv / (rv + rh), rv and rh   */
/*   the columns and rows still to cross: u(rv + rh) < rv), and each   */
/*   move opens one cell of the river it crosses, uniform along the    */
/*   current room's side (position drawn right after the move).        */
/* DistShift(S, k): goal (S-2, 1); lava on rows 1 and r2 (r2 = 2 for   */
/*   k = 1, S - 2 for k = 2) over columns 3..S-3; no random draws.     */
/* Dynamic-Obstacles(S, n): goal (S-2, S-2); n blue balls, ball b at   */
/*   the k-th empty interior cell other than the agent's, k uniform,    */
/*   placed in order b = 0..n-1; their positions are listed in obst     */
/*   (x, y per ball, 0xFF for unused slots and other families).         */
/* GoToDoor(S): a room of width w = 5 + u(S-4) and height             */
/*   h = 5 + u(S-4) in the top-left corner, walled; every cell outside  */
/*   the room is wall too.  One closed door on each room wall, at a     */
/*   uniform non-corner position, drawn in the order top (x), right     */
/*   (y), bottom (x), left (y); the four doors take four distinct       */
/*   colours by a partial Fisher-Yates shuffle of the six (step k swaps */
/*   colour k with colour k + u(6-k)), door i getting colour i of the   */
/*   shuffle; the mission is the colour of door u(4) (kept in obst[0]); */
/*   agent uniform over the room's interior; direction uniform.  No     */
/*   goal.                                                              */
/* KeyCorridor(S = 3s-2, R rows): a lattice of 3 x R rooms of size s    */
/*   (walls shared, stride s-1) in the top rows of the grid, H = R(s-1) */
/*   + 1; the rows below H are wall.  The middle column is a hallway:   */
/*   the walls between its rooms are open.  Every wall between two     */
/*   rooms has a door position, drawn in the order rows j, columns i:   */
/*   the right wall of room (i, j) (i < 2), then its lower wall (j <    */
/*   R-1), each uniform over the wall's s-2 inner cells.  Then: the     */
/*   locked room's row u(R) and the colour u(6) of its locked door, on  */
/*   the wall between the hallway and the right-column room of that     */
/*   row; the goal uniform in that room; the key (the door's colour) in */
/*   the left-column room of row u(R), uniform; the agent uniform in    */
/*   the hallway room of row R/2, heading uniform.  Last, every room is */
/*   connected as MiniGrid's connect_all does: while some room is not   */
/*   reachable from the agent's room through openings and doors, draw a */
/*   room (u(3), u(R)) and a side u(4); if a neighbour lies there, the  */
/*   wall between has no door or opening yet and neither room is the   */
/*   locked one, add a closed door of colour u(6) at the wall's         */
/*   position (at most 1024 draws of a room).  The paper lists R1 (the  */
/*   goal square) for this family, so the goal sits behind the locked   */
/*   door where MiniGrid puts a ball to pick up.                        */
/* Pinned by: structural invariants, uniformity tests and the hand     */
/* layouts in tests; agreement with MiniGrid's own generators: parity  */
/* unpinned (MiniGrid is not available).                               */
/* ------------------------------------------------------------------ */
static void crossings(uint8_t *grid, int S, int N, uint64_t seed,
                      uint32_t rng_id, uint32_t episode, uint32_t *w);

int ox_layout(int family, int S, int param, uint64_t seed, uint32_t rng_id,
              uint32_t episode, uint8_t *grid, int *ax, int *ay, int *adir,
              uint8_t *obst) {
  if (!ox_side_ok(family, S, param)) return -1;
  if (obst) memset(obst, 0xFF, 2 * OX_MAX_OBST);
  uint32_t w = 0;
#define DRAW(n) ox_uniform(layout_word(seed, rng_id, episode, w++), (uint32_t)(n))
  for (int y = 0; y < S; ++y)
    for (int x = 0; x < S; ++x) {
      int border = (x == 0 || y == 0 || x == S - 1 || y == S - 1);
      if (border) put(grid, S, x, y, O_WALL, C_GREY, 0);
      else put(grid, S, x, y, O_EMPTY, 0, 0);
    }
  if (family == FAM_EMPTY) {
    put(grid, S, S - 2, S - 2, O_GOAL, C_GREEN, 0);
    uint32_t n = count_empty(grid, S, 1, S - 2, 1, S - 2);
    if (kth_empty(grid, S, 1, S - 2, 1, S - 2, DRAW(n), ax, ay)) return -2;
    *adir = (int)DRAW(4);
  } else if (family == FAM_TWOROOM) {
    int c = 2 + (int)DRAW(S - 4);
    int d = 1 + (int)DRAW(S - 3);
    int colour = (int)DRAW(6);
    for (int y = 0; y < S; ++y) put(grid, S, c, y, O_WALL, C_GREY, 0);
    put(grid, S, c, d, O_DOOR, colour, D_LOCKED);
    put(grid, S, S - 2, S - 2, O_GOAL, C_GREEN, 0);
    int kx, ky;
    uint32_t n = count_empty(grid, S, 1, c - 1, 1, S - 2);
    if (kth_empty(grid, S, 1, c - 1, 1, S - 2, DRAW(n), &kx, &ky)) return -2;
    put(grid, S, kx, ky, O_KEY, colour, 0);
    n = count_empty(grid, S, 1, c - 1, 1, S - 2);
    if (kth_empty(grid, S, 1, c - 1, 1, S - 2, DRAW(n), ax, ay)) return -2;
    *adir = (int)DRAW(4);
  } else if (family == FAM_FOURROOMS) {
    int m = S / 2;
    for (int i = 0; i < S; ++i) {
      put(grid, S, m, i, O_WALL, C_GREY, 0);
      put(grid, S, i, m, O_WALL, C_GREY, 0);
    }
    int g1 = 1 + (int)DRAW(m - 1);
    int g2 = m + 1 + (int)DRAW(m - 1);
    int g3 = 1 + (int)DRAW(m - 1);
    int g4 = m + 1 + (int)DRAW(m - 1);
    put(grid, S, m, g1, O_EMPTY, 0, 0);
    put(grid, S, m, g2, O_EMPTY, 0, 0);
    put(grid, S, g3, m, O_EMPTY, 0, 0);
    put(grid, S, g4, m, O_EMPTY, 0, 0);
    int gx, gy;
    uint32_t n = count_empty(grid, S, 1, S - 2, 1, S - 2);
    if (kth_empty(grid, S, 1, S - 2, 1, S - 2, DRAW(n), &gx, &gy)) return -2;
    put(grid, S, gx, gy, O_GOAL, C_GREEN, 0);
    n = count_empty(grid, S, 1, S - 2, 1, S - 2);
    if (kth_empty(grid, S, 1, S - 2, 1, S - 2, DRAW(n), ax, ay)) return -2;
    *adir = (int)DRAW(4);
  } else if (family == FAM_KEYCORRIDOR) {
    const int rs = (S + 2) / 3, st = rs - 1, R = param, H = R * st + 1;
    for (int y = 0; y < S; ++y)
      for (int x = 0; x < S; ++x)
        if (y >= H || x % st == 0 || y % st == 0) put(grid, S, x, y, O_WALL, C_GREY, 0);
    /* door positions of the walls between rooms: pv[i][j] between (i, j)
     * and (i+1, j), ph[i][j] between (i, j) and (i, j+1) */
    int pv[2][3], ph[3][2];
    for (int j = 0; j < R; ++j)
      for (int i = 0; i < 3; ++i) {
        if (i < 2) pv[i][j] = (int)DRAW(rs - 2);
        if (j < R - 1) ph[i][j] = (int)DRAW(rs - 2);
      }
    /* openings: ov[i][j] / oh[i][j] = 1 where the wall is open or has a door */
    int ov[2][3] = {{0}}, oh[3][2] = {{0}};
    for (int j = 0; j + 1 < R; ++j) {           /* the hallway */
      oh[1][j] = 1;
      for (int x = st + 1; x < 2 * st; ++x) put(grid, S, x, (j + 1) * st, O_EMPTY, 0, 0);
    }
    int rl = (int)DRAW(R);
    int colour = (int)DRAW(6);
    put(grid, S, 2 * st, rl * st + 1 + pv[1][rl], O_DOOR, colour, D_LOCKED);
    ov[1][rl] = 1;
    int gx, gy, kx, ky;
    uint32_t n = count_empty(grid, S, 2 * st + 1, 3 * st - 1, rl * st + 1, (rl + 1) * st - 1);
    if (kth_empty(grid, S, 2 * st + 1, 3 * st - 1, rl * st + 1, (rl + 1) * st - 1, DRAW(n), &gx, &gy))
      return -2;
    put(grid, S, gx, gy, O_GOAL, C_GREEN, 0);
    int rk = (int)DRAW(R);
    n = count_empty(grid, S, 1, st - 1, rk * st + 1, (rk + 1) * st - 1);
    if (kth_empty(grid, S, 1, st - 1, rk * st + 1, (rk + 1) * st - 1, DRAW(n), &kx, &ky)) return -2;
    put(grid, S, kx, ky, O_KEY, colour, 0);
    int ra = R / 2;
    n = count_empty(grid, S, st + 1, 2 * st - 1, ra * st + 1, (ra + 1) * st - 1);
    if (kth_empty(grid, S, st + 1, 2 * st - 1, ra * st + 1, (ra + 1) * st - 1, DRAW(n), ax, ay))
      return -2;
    *adir = (int)DRAW(4);
    for (int it = 0; it < 1024; ++it) {
      /* rooms reachable from the agent's: repeated relaxation over the walls */
      int reach[3][3] = {{0}}, grew = 1, count = 0;
      reach[1][ra] = 1;
      while (grew) {
        grew = 0;
        for (int j = 0; j < R; ++j)
          for (int i = 0; i < 3; ++i) {
            if (reach[i][j]) continue;
            int nb = (i > 0 && ov[i - 1][j] && reach[i - 1][j]) || (i < 2 && ov[i][j] && reach[i + 1][j]) ||
                     (j > 0 && oh[i][j - 1] && reach[i][j - 1]) || (j < R - 1 && oh[i][j] && reach[i][j + 1]);
            if (nb) { reach[i][j] = 1; grew = 1; }
          }
      }
      for (int j = 0; j < R; ++j)
        for (int i = 0; i < 3; ++i) count += reach[i][j];
      if (count == 3 * R) break;
      int i = (int)DRAW(3), j = (int)DRAW(R), k = (int)DRAW(4);
      int i2 = i + (k == 0) - (k == 2), j2 = j + (k == 1) - (k == 3);
      if (i2 < 0 || i2 > 2 || j2 < 0 || j2 >= R) continue;
      int *open = (j2 == j) ? &ov[i < i2 ? i : i2][j] : &oh[i][j < j2 ? j : j2];
      if (*open) continue;
      if ((i == 2 && j == rl) || (i2 == 2 && j2 == rl)) continue;
      int c = (int)DRAW(6);
      *open = 1;
      if (j2 == j) {
        int iw = i < i2 ? i : i2;
        put(grid, S, (iw + 1) * st, j * st + 1 + pv[iw][j], O_DOOR, c, D_CLOSED);
      } else {
        int jw = j < j2 ? j : j2;
        put(grid, S, i * st + 1 + ph[i][jw], (jw + 1) * st, O_DOOR, c, D_CLOSED);
      }
    }
  } else if (family == FAM_GOTODOOR) {
    int rw = 5 + (int)DRAW(S - 4);
    int rh = 5 + (int)DRAW(S - 4);
    for (int y = 0; y < S; ++y)
      for (int x = 0; x < S; ++x)
        if (x >= rw - 1 || y >= rh - 1) put(grid, S, x, y, O_WALL, C_GREY, 0);
    int dx[4], dy[4];
    dx[0] = 1 + (int)DRAW(rw - 2); dy[0] = 0;        /* top */
    dx[1] = rw - 1; dy[1] = 1 + (int)DRAW(rh - 2);   /* right */
    dx[2] = 1 + (int)DRAW(rw - 2); dy[2] = rh - 1;   /* bottom */
    dx[3] = 0; dy[3] = 1 + (int)DRAW(rh - 2);        /* left */
    int col[6] = {0, 1, 2, 3, 4, 5};
    for (int k = 0; k < 4; ++k) {
      int r = k + (int)DRAW(6 - k);
      int tmp = col[k]; col[k] = col[r]; col[r] = tmp;
    }
    for (int i = 0; i < 4; ++i) put(grid, S, dx[i], dy[i], O_DOOR, col[i], D_CLOSED);
    int target = (int)DRAW(4);
    if (obst) obst[0] = (uint8_t)col[target];
    uint32_t n = count_empty(grid, S, 1, rw - 2, 1, rh - 2);
    if (kth_empty(grid, S, 1, rw - 2, 1, rh - 2, DRAW(n), ax, ay)) return -2;
    *adir = (int)DRAW(4);
  } else {
    *ax = 1; *ay = 1; *adir = 0;
    if (family == FAM_LAVAGAP) {
      put(grid, S, S - 2, S - 2, O_GOAL, C_GREEN, 0);
      int c = 2 + (int)DRAW(S - 4);
      int gap = 1 + (int)DRAW(S - 2);
      for (int y = 1; y <= S - 2; ++y)
        if (y != gap) put(grid, S, c, y, O_LAVA, C_RED, 0);
    } else if (family == FAM_CROSSINGS) {
      put(grid, S, S - 2, S - 2, O_GOAL, C_GREEN, 0);
      crossings(grid, S, param, seed, rng_id, episode, &w);
    } else if (family == FAM_DYNOBS) {
      put(grid, S, S - 2, S - 2, O_GOAL, C_GREEN, 0);
      for (int b = 0; b < param; ++b) {
        /* empty interior cells other than the agent's (1, 1), row-major */
        uint32_t n = count_empty(grid, S, 1, S - 2, 1, S - 2) - 1u;
        uint32_t k = DRAW(n) + 1u;   /* skip the agent's cell, the first empty one */
        int bx, by;
        if (kth_empty(grid, S, 1, S - 2, 1, S - 2, k, &bx, &by)) return -2;
        put(grid, S, bx, by, O_BALL, C_BLUE, 0);
        if (obst) { obst[2 * b] = (uint8_t)bx; obst[2 * b + 1] = (uint8_t)by; }
      }
    } else {
      put(grid, S, S - 2, 1, O_GOAL, C_GREEN, 0);
      int r2 = param == 1 ? 2 : S - 2;
      for (int x = 3; x <= S - 3; ++x) {
        put(grid, S, x, 1, O_LAVA, C_RED, 0);
        put(grid, S, x, r2, O_LAVA, C_RED, 0);
      }
    }
  }
#undef DRAW
  return 0;
}

/* Crossings(S, N) body: draws continue the layout stream at word *w. */
static void crossings(uint8_t *grid, int S, int N, uint64_t seed,
                      uint32_t rng_id, uint32_t episode, uint32_t *w) {
#define DRAW(n) ox_uniform(layout_word(seed, rng_id, episode, (*w)++), (uint32_t)(n))
  /* candidates: columns 2, 4, .., S-3 (coded as +x), then rows (coded -y) */
  int cand[32], M = 0;
  for (int x = 2; x <= S - 3; x += 2) cand[M++] = x;
  for (int y = 2; y <= S - 3; y += 2) cand[M++] = -y;
  for (int k = 0; k < N; ++k) {
    int r = k + (int)DRAW(M - k);
    int tmp = cand[k]; cand[k] = cand[r]; cand[r] = tmp;
  }
  /* the chosen columns and rows, ascending, framed by the border */
  int vlim[34], hlim[34], nv = 0, nh = 0;
  vlim[0] = 0; hlim[0] = 0;
  for (int v = 1; v <= S - 2; ++v)
    for (int k = 0; k < N; ++k) {
      if (cand[k] == v) vlim[++nv] = v;
      if (cand[k] == -v) hlim[++nh] = v;
    }
  vlim[nv + 1] = S - 1; hlim[nh + 1] = S - 1;
  for (int i = 1; i <= nv; ++i)
    for (int y = 1; y <= S - 2; ++y) put(grid, S, vlim[i], y, O_LAVA, C_RED, 0);
  for (int j = 1; j <= nh; ++j)
    for (int x = 1; x <= S - 2; ++x) put(grid, S, x, hlim[j], O_LAVA, C_RED, 0);
  /* the path: room (ci, rj) starts at (0, 0) and ends at (nv, nh) */
  int ci = 0, rj = 0;
  for (int q = 0; q < N; ++q) {
    int rv = nv - ci, rh = nh - rj;
    int east = (int)DRAW(rv + rh) < rv;
    if (east) {
      int lo = hlim[rj], hi = hlim[rj + 1];
      int y = lo + 1 + (int)DRAW(hi - lo - 1);
      put(grid, S, vlim[ci + 1], y, O_EMPTY, 0, 0);
      ci += 1;
    } else {
      int lo = vlim[ci], hi = vlim[ci + 1];
      int x = lo + 1 + (int)DRAW(hi - lo - 1);
      put(grid, S, x, hlim[rj + 1], O_EMPTY, 0, 0);
      rj += 1;
    }
  }
#undef DRAW
}

/* ------------------------------------------------------------------ */
/* Observation system O: S -> O, symbolic_first_person with R = 7     */
/* (Table "observations"), following MiniGrid's partial view because  */
/* the environments match MiniGrid (Sec. 3.2.1):                      */
/*  1. the 7x7 view, agent at view column 3, row 6, facing row 0:     */
/*     world(i, j) = agent + (i-3) * right + (6-j) * forward, with    */
/*     right = (-forward_y, forward_x); cells outside the grid are    */
/*     walls;                                                          */
/*  2. occlusion: walls and non-open doors block sight.  Row by row   */
/*     from the agent's row (6) to the farthest (0): a left-to-right  */
/*     pass, then a right-to-left pass, over visible see-through cells*/
/*     which make their row neighbour and the two cells ahead visible;*/
/*  3. encoding: invisible cells (0,0,0); visible cells their         */
/*     (type, colour, state); the agent's own cell shows what it      */
/*     carries, or an empty cell (1,0,0) for an empty hand.           */
/* Output layout obs[j][i][c]: row j (0 = farthest), column i         */
/* (0 = the agent's left), channel c.                                  */
/* Pinned by the hand-worked views in tests/golden/ and by rotation    */
/* invariance; agreement with MiniGrid itself: parity unpinned.        */
/* ------------------------------------------------------------------ */
void ox_observe(const uint8_t *grid, int S, int ax, int ay, int dir,
                int32_t carry, uint8_t *obs /* [7][7][3] */) {
  uint8_t view[OX_VIEW][OX_VIEW][3]; /* [i][j][c] */
  int see[OX_VIEW][OX_VIEW];
  int vis[OX_VIEW][OX_VIEW];
  int fx = DIR_X[dir], fy = DIR_Y[dir];
  int rx = -fy, ry = fx;
  for (int i = 0; i < OX_VIEW; ++i)
    for (int j = 0; j < OX_VIEW; ++j) {
      int wx = ax + (i - 3) * rx + (6 - j) * fx;
      int wy = ay + (i - 3) * ry + (6 - j) * fy;
      if (wx < 0 || wy < 0 || wx >= S || wy >= S) {
        view[i][j][0] = O_WALL; view[i][j][1] = C_GREY; view[i][j][2] = 0;
      } else {
        const uint8_t *c = grid + 3 * (wy * S + wx);
        view[i][j][0] = c[0]; view[i][j][1] = c[1]; view[i][j][2] = c[2];
      }
      int type = view[i][j][0];
      int opaque = (type == O_WALL) || (type == O_DOOR && view[i][j][2] != D_OPEN);
      see[i][j] = !opaque;
      vis[i][j] = 0;
    }
  vis[3][6] = 1;
  for (int j = OX_VIEW - 1; j >= 0; --j) {
    for (int i = 0; i < OX_VIEW - 1; ++i) {
      if (!vis[i][j] || !see[i][j]) continue;
      vis[i + 1][j] = 1;
      if (j > 0) { vis[i + 1][j - 1] = 1; vis[i][j - 1] = 1; }
    }
    for (int i = OX_VIEW - 1; i >= 1; --i) {
      if (!vis[i][j] || !see[i][j]) continue;
      vis[i - 1][j] = 1;
      if (j > 0) { vis[i - 1][j - 1] = 1; vis[i][j - 1] = 1; }
    }
  }
  for (int j = 0; j < OX_VIEW; ++j)
    for (int i = 0; i < OX_VIEW; ++i) {
      uint8_t *o = obs + 3 * (j * OX_VIEW + i);
      if (i == 3 && j == 6) {
        o[0] = (uint8_t)(carry & 0xFF);
        o[1] = (uint8_t)((carry >> 8) & 0xFF);
        o[2] = (uint8_t)((carry >> 16) & 0xFF);
      } else if (vis[i][j]) {
        o[0] = view[i][j][0]; o[1] = view[i][j][1]; o[2] = view[i][j][2];
      } else {
        o[0] = 0; o[1] = 0; o[2] = 0;
      }
    }
}

/* categorical_first_person (Table "observations"): the entity-id grid  */
/* of the same 7x7 view, [j][i], one byte per cell: the type index of a  */
/* visible cell, 0 where unseen; the agent's cell shows the carried      */
/* object's type (1 for an empty hand).  Pinned by the type channels of  */
/* the hand-worked views in tests/golden/.                               */
void ox_observe_categorical(const uint8_t *grid, int S, int ax, int ay, int dir,
                            int32_t carry, uint8_t *obs /* [7][7] */) {
  uint8_t sym[OX_VIEW * OX_VIEW * 3];
  ox_observe(grid, S, ax, ay, dir, carry, sym);
  for (int k = 0; k < OX_VIEW * OX_VIEW; ++k) obs[k] = sym[3 * k];
}

/* symbolic (Table "observations"): the whole grid in the canonical      */
/* encoding, [S][S][3] in the grid's own layout, with the agent drawn on */
/* its cell as (agent 10, red 0, heading), the way MiniGrid encodes a    */
/* fully observed grid; what the agent carries is not shown.  Pinned by  */
/* the hand-worked grid in tests/golden/ and by agreement with the       */
/* first-person view at every visible cell.                              */
void ox_observe_full(const uint8_t *grid, int S, int ax, int ay, int dir,
                     uint8_t *obs /* [S][S][3] */) {
  for (int y = 0; y < S; ++y)
    for (int x = 0; x < S; ++x) {
      const uint8_t *c = grid + 3 * (y * S + x);
      uint8_t *o = obs + 3 * (y * S + x);
      if (x == ax && y == ay) {
        o[0] = O_AGENT; o[1] = C_RED; o[2] = (uint8_t)dir;
      } else {
        o[0] = c[0]; o[1] = c[1]; o[2] = c[2];
      }
    }
}

/* categorical (Table "observations"): the entity-id grid [S][S], one    */
/* byte per cell: the type index of every cell, the agent's cell 10.     */
/* Pinned like the symbolic grid above.                                  */
void ox_observe_full_categorical(const uint8_t *grid, int S, int ax, int ay, int dir,
                                 uint8_t *obs /* [S][S] */) {
  (void)dir;
  for (int y = 0; y < S; ++y)
    for (int x = 0; x < S; ++x)
      obs[y * S + x] = (x == ax && y == ay) ? (uint8_t)O_AGENT : grid[3 * (y * S + x)];
}

/* ------------------------------------------------------------------ */
/* rgb and rgb_first_person (Table "observations": images of 32 pixels */
/* per cell side, [32H][32W][3] of the whole grid and [32R][32R][3] of */
/* the first-person view).  Every entity carries a sprite, a          */
/* u8[32][32][3] image (Table "components": HasSprite); the sprites are */
/* data, an atlas of 264 images indexed (type * 6 + colour) * 4 +      */
/* state for type 0..10, colour 0..5, state 0..3 (a door's state, the  */
/* agent's heading).  A cell is drawn as the sprite of its symbolic     */
/* triple; a triple outside those ranges draws sprite 0, the unseen     */
/* cell's.  The image of W x W cells is [32W][32W][3]: pixel row        */
/* 32 j + py, column 32 i + px holds pixel (py, px) of cell (i, j)'s    */
/* sprite.  rgb draws the symbolic whole grid (the agent over its cell */
/* with its heading); rgb_first_person draws the first-person view      */
/* with the agent's own cell as the agent facing the top of the image  */
/* (heading 3, north), the carried object not drawn.                   */
/* Pinned by decoding: under an atlas whose pixels spell out their      */
/* sprite index and position, every pixel names its cell's triple in   */
/* the independently pinned symbolic views.  Agreement with NAVIX's or  */
/* MiniGrid's drawings: parity unpinned (their sprites are not here).   */
/* ------------------------------------------------------------------ */
#define OX_SPRITE 32
#define OX_SPRITE_BYTES (OX_SPRITE * OX_SPRITE * 3)

static int sprite_index(const uint8_t *triple) {
  if (triple[0] > O_AGENT || triple[1] > C_GREY || triple[2] > 3) return 0;
  return (triple[0] * 6 + triple[1]) * 4 + triple[2];
}

/* Draw W x W cells (symbolic triples, [W][W][3]) into img [32W][32W][3]. */
void ox_render(const uint8_t *cells, int W, const uint8_t *sprites, uint8_t *img) {
  const size_t row_pixels = (size_t)OX_SPRITE * (size_t)W;
  for (int j = 0; j < W; ++j)
    for (int i = 0; i < W; ++i) {
      const uint8_t *sp = sprites + (size_t)sprite_index(cells + 3 * (j * W + i)) * OX_SPRITE_BYTES;
      for (int py = 0; py < OX_SPRITE; ++py)
        for (int px = 0; px < OX_SPRITE; ++px)
          for (int ch = 0; ch < 3; ++ch) {
            size_t row = (size_t)(OX_SPRITE * j + py), col = (size_t)(OX_SPRITE * i + px);
            img[(row * row_pixels + col) * 3 + ch] = sp[(py * OX_SPRITE + px) * 3 + ch];
          }
    }
}

void ox_observe_rgb(const uint8_t *grid, int S, int ax, int ay, int dir,
                    const uint8_t *sprites, uint8_t *img /* [224][224][3] */) {
  uint8_t view[OX_VIEW * OX_VIEW * 3];
  ox_observe(grid, S, ax, ay, dir, O_EMPTY, view);
  uint8_t *agent = view + 3 * ((OX_VIEW - 1) * OX_VIEW + 3);
  agent[0] = O_AGENT; agent[1] = C_RED; agent[2] = 3;
  ox_render(view, OX_VIEW, sprites, img);
}

void ox_observe_rgb_full(const uint8_t *grid, int S, int ax, int ay, int dir,
                         const uint8_t *sprites, uint8_t *img /* [32S][32S][3] */) {
  uint8_t whole[32 * 32 * 3];
  if (S > 32) return;
  ox_observe_full(grid, S, ax, ay, dir, whole);
  ox_render(whole, S, sprites, img);
}

/* Observation modes: 0 symbolic_first_person, 1 categorical_first_person, */
/* 2 symbolic, 3 categorical, 4 rgb_first_person, 5 rgb.  The first-person */
/* records of one output row are [N][147], [N][49] or [N][224][224][3];    */
/* the whole-grid records are packed like the grids, env i's at            */
/* grid_off(i) (symbolic), grid_off(i) / 3 (categorical) or 1024           */
/* grid_off(i) (rgb) of a row of sum 3 S^2, sum S^2 or sum 3072 S^2 bytes. */
static void emit_obs(int mode, const uint8_t *sprites, const uint8_t *grid, int S, int ax,
                     int ay, int dir, int32_t carry, uint8_t *obs) {
  if (mode == 1) ox_observe_categorical(grid, S, ax, ay, dir, carry, obs);
  else if (mode == 2) ox_observe_full(grid, S, ax, ay, dir, obs);
  else if (mode == 3) ox_observe_full_categorical(grid, S, ax, ay, dir, obs);
  else if (mode == 4) ox_observe_rgb(grid, S, ax, ay, dir, sprites, obs);
  else if (mode == 5) ox_observe_rgb_full(grid, S, ax, ay, dir, sprites, obs);
  else ox_observe(grid, S, ax, ay, dir, carry, obs);
}

/* ------------------------------------------------------------------ */
/* Reward R (Sec. 3.2.1, Eq. (1); Table "rewards", on_goal_reached),  */
/* in fp32, three separately rounded operations:                       */
/*   q = t / T, p = 0.9 * q, r = 1 - p  (t counted after this step).   */
/* reward_mode 1 is the Markovian unit reward the paper uses instead.  */
/* Pinned by the exact rational 1 - 9t/(10T) within fp32 error bounds. */
/* ------------------------------------------------------------------ */
float ox_goal_reward(int32_t t, int32_t T, int reward_mode) {
  if (reward_mode == 1) return 1.0f;
  volatile float q = (float)t / (float)T;
  volatile float p = 0.9f * q;
  volatile float r = 1.0f - p;
  return r;
}

/* one env of a batch */
typedef struct {
  uint8_t *grid;
  int32_t *x, *y, *dir, *t, *carry;
  uint32_t *episode;
  uint8_t *done_prev;
  uint32_t *calls;
  uint8_t *obst;   /* 16 bytes: obstacle positions (Dynamic-Obstacles) */
} ox_env_ref;

static int is_pickable(int type) {
  return type == O_KEY || type == O_BALL || type == O_BOX;
}

/* ------------------------------------------------------------------ */
/* Transition system of Dynamic-Obstacles (Table "systems"; Fig. 1):  */
/* each ball, in list order, moves to a uniformly drawn empty cell of */
/* the 8 around it that the agent does not occupy, drawn as the k-th  */
/* such cell in row-major order, k = u(count) of its word; with no    */
/* such cell it stays.  Ball b's word: key = seed, counter = (rng_id, */
/* call, b / 4, 2), lane b % 4, call = the env's step-call count.     */
/* A list entry off the interior (a malformed state) does not move.   */
/* Pinned by hand-worked moves, uniformity and invariant tests.       */
/* ------------------------------------------------------------------ */
static void move_obstacles(uint8_t *grid, int S, int n, int ax, int ay,
                           uint8_t *obst, uint64_t seed, uint32_t rng_id,
                           uint32_t call) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int b = 0; b < n; ++b) {
    uint32_t ctr[4] = {rng_id, call, (uint32_t)(b / 4), 2u}, out[4];
    ox_philox4x32_10(ctr, key, out);
    uint32_t word = out[b % 4];
    int bx = obst[2 * b], by = obst[2 * b + 1];
    int cx[8], cy[8], count = 0;
    if (bx < 1 || by < 1 || bx > S - 2 || by > S - 2) continue;   /* malformed entry */
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int x = bx + dx, y = by + dy;
        if ((dx == 0 && dy == 0) || (x == ax && y == ay)) continue;
        if (cell(grid, S, x, y)[0] != O_EMPTY) continue;
        cx[count] = x; cy[count] = y; ++count;
      }
    if (count == 0) continue;
    uint32_t k = ox_uniform(word, (uint32_t)count);
    put(grid, S, bx, by, O_EMPTY, 0, 0);
    put(grid, S, cx[k], cy[k], O_BALL, C_BLUE, 0);
    obst[2 * b] = (uint8_t)cx[k];
    obst[2 * b + 1] = (uint8_t)cy[k];
  }
}

/* ------------------------------------------------------------------ */
/* One environment step: the interaction protocol of Sec. 3.2.2 with  */
/* autoreset.  If the previous step ended the episode, this call      */
/* ignores its action and returns the first timestep of the next      */
/* episode (reset pads: action -1 recorded as 0xFF, reward 0).        */
/* Otherwise: intervention I(s, a) (turn, forward with collision,     */
/* pickup, drop, toggle with colour-matched keys; App. A), transition */
/* (identity except in Dynamic-Obstacles), observation O(s'), reward  */
/* R, and termination (goal reached or lava entered) plus truncation   */
/* at t = T.                                                           */
/* Lava (Table "entities") is walked onto like an empty cell and ends  */
/* the episode with reward -1 (R2 of Table "envs"; on_lava_fall of     */
/* Tables "rewards" and "terminations"), in both reward modes: the     */
/* time discount of Eq. (1) applies to the goal reward only.           */
/* Dynamic-Obstacles (R3): the env has three actions (any other acts   */
/* as turn left); the cell ahead is checked first, then the balls     */
/* move (the transition system), then the action applies; moving       */
/* forward when that cell held a ball or a wall ends the episode with  */
/* reward -1, as MiniGrid's version does.                              */
/* GoToDoor (on_door_done of Tables "rewards" and "terminations"): the */
/* done action (any action >= 6) with the cell ahead a door of the     */
/* mission's colour ends the episode with the goal reward; toggling    */
/* (the door opens or closes as usual) ends it with reward 0, as       */
/* MiniGrid's version does.                                            */
/* ------------------------------------------------------------------ */
static void step_one(int family, int S, int param, int32_t T, uint64_t seed,
                     uint32_t rng_id, int reward_mode, int obs_mode,
                     const uint8_t *sprites, ox_env_ref e,
                     uint32_t action, uint8_t *obs, float *reward,
                     uint8_t *flags, uint8_t *rec_action) {
  if (*e.done_prev) {
    *e.episode += 1u;
    ox_layout(family, S, param, seed, rng_id, *e.episode, e.grid, e.x, e.y,
              e.dir, e.obst);
    *e.t = 0;
    *e.carry = O_EMPTY;
    *e.done_prev = 0;
    if (obs) emit_obs(obs_mode, sprites, e.grid, S, *e.x, *e.y, *e.dir, *e.carry, obs);
    *reward = 0.0f;
    *flags = OX_FLAG_FIRST;
    *rec_action = OX_ACTION_NONE;
    return;
  }
  int dir = *e.dir;
  int fx = *e.x + DIR_X[dir], fy = *e.y + DIR_Y[dir];
  uint8_t *front = cell(e.grid, S, fx, fy);
  int terminated = 0, lava = 0, blocked = 0;
  int goal = 0;   /* the task is achieved: the goal reached, or the mission's door done */
  if (family == FAM_DYNOBS) {
    if (action > A_FORWARD) action = A_LEFT;   /* three actions only */
    blocked = front[0] != O_EMPTY && front[0] != O_GOAL;
    move_obstacles(e.grid, S, param, *e.x, *e.y, e.obst, seed, rng_id, *e.calls);
  }
  switch (action) {
    case A_LEFT: *e.dir = (dir + 3) % 4; break;
    case A_RIGHT: *e.dir = (dir + 1) % 4; break;
    case A_FORWARD: {
      int type = front[0];
      int walkable = type == O_EMPTY || type == O_GOAL || type == O_LAVA ||
                     (type == O_DOOR && front[2] == D_OPEN);
      if (walkable) { *e.x = fx; *e.y = fy; }
      if (type == O_GOAL) terminated = goal = 1;
      if (type == O_LAVA) terminated = lava = 1;
      break;
    }
    case A_PICKUP:
      if (*e.carry == O_EMPTY && is_pickable(front[0])) {
        *e.carry = front[0] | (front[1] << 8) | (front[2] << 16);
        front[0] = O_EMPTY; front[1] = 0; front[2] = 0;
      }
      break;
    case A_DROP:
      if (*e.carry != O_EMPTY && front[0] == O_EMPTY) {
        front[0] = (uint8_t)(*e.carry & 0xFF);
        front[1] = (uint8_t)((*e.carry >> 8) & 0xFF);
        front[2] = (uint8_t)((*e.carry >> 16) & 0xFF);
        *e.carry = O_EMPTY;
      }
      break;
    case A_TOGGLE:
      if (front[0] == O_DOOR) {
        if (front[2] == D_LOCKED) {
          int carry_type = *e.carry & 0xFF, carry_colour = (*e.carry >> 8) & 0xFF;
          if (carry_type == O_KEY && carry_colour == front[1]) front[2] = D_OPEN;
        } else {
          front[2] = front[2] == D_OPEN ? D_CLOSED : D_OPEN;
        }
      }
      if (family == FAM_GOTODOOR) terminated = 1;   /* toggling ends GoToDoor, reward 0 */
      break;
    default: /* done, and any out-of-range action: no effect on the grid */
      if (family == FAM_GOTODOOR && front[0] == O_DOOR && front[1] == e.obst[0])
        terminated = goal = 1;                      /* on_door_done */
      break;
  }
  *e.t += 1;
  int truncated = *e.t >= T;
  if (blocked && action == A_FORWARD) terminated = lava = 1;
  if (lava) *reward = -1.0f;
  else *reward = goal ? ox_goal_reward(*e.t, T, reward_mode) : 0.0f;
  *flags = (uint8_t)((terminated ? OX_FLAG_TERMINATED : 0) |
                     (truncated ? OX_FLAG_TRUNCATED : 0));
  *rec_action = (uint8_t)action;
  *e.done_prev = (uint8_t)(terminated || truncated);
  if (obs) emit_obs(obs_mode, sprites, e.grid, S, *e.x, *e.y, *e.dir, *e.carry, obs);
}

/* ------------------------------------------------------------------ */
/* Batch entry points (SoA, host memory).  Per env i:                  */
/*   family[i], side[i], param[i], max_steps[i], seed[i], rng_id[i],  */
/*   grid + grid_off[i] ([side][side][3]),                             */
/*   x, y, dir, t, carry, episode, done_prev.                          */
/* Outputs are [N] rows; obs records as emit_obs describes; obs and    */
/* mission may be NULL.                                                */
/* nthreads > 0 runs envs in parallel with OpenMP (timing mode).       */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t n;
  const uint8_t *family, *side;
  const int32_t *max_steps;
  const uint64_t *seed;
  const uint32_t *rng_id;
  const uint64_t *grid_off;
  int32_t reward_mode;
  const uint8_t *param;   /* per env family parameter, or NULL (all 0) */
  int32_t obs_mode;       /* 0 symbolic_first_person, 1 categorical_first_person,
                             2 symbolic, 3 categorical, 4 rgb_first_person, 5 rgb */
  const uint8_t *sprites; /* modes 4 and 5: the atlas [264][32][32][3] */
} ox_batch;

typedef struct {
  uint8_t *grid;
  int32_t *x, *y, *dir, *t, *carry;
  uint32_t *episode;
  uint8_t *done_prev;
  uint32_t *calls;   /* step calls since reset (the random policy's counter) */
  uint8_t *obst;     /* [N][16] obstacle positions (x, y per ball, 0xFF unused) */
} ox_state;

#define PARAM(b, i) ((b)->param ? (int)(b)->param[i] : 0)

/* bytes of one output row of observations */
static size_t obs_row_bytes(const ox_batch *b) {
  if (b->obs_mode == 0 || b->obs_mode == 1) return (size_t)b->n * (b->obs_mode == 1 ? 49 : 147);
  if (b->obs_mode == 4) return (size_t)b->n * 147 * 1024;
  size_t cells = 0;
  for (int i = 0; i < b->n; ++i) cells += (size_t)b->side[i] * b->side[i];
  return b->obs_mode == 2 ? 3 * cells : b->obs_mode == 5 ? 3072 * cells : cells;
}

/* env i's record in output row `row` */
static uint8_t *obs_at(const ox_batch *b, uint8_t *obs, size_t row_bytes, size_t row, int i) {
  uint8_t *r = obs + row * row_bytes;
  switch (b->obs_mode) {
    case 1: return r + (size_t)49 * i;
    case 2: return r + b->grid_off[i];
    case 3: return r + b->grid_off[i] / 3;
    case 4: return r + (size_t)147 * 1024 * i;
    case 5: return r + (size_t)1024 * b->grid_off[i];
    default: return r + (size_t)147 * i;
  }
}

static ox_env_ref env_ref(const ox_batch *b, const ox_state *s, int i) {
  ox_env_ref e;
  e.grid = s->grid + b->grid_off[i];
  e.x = s->x + i; e.y = s->y + i; e.dir = s->dir + i; e.t = s->t + i;
  e.carry = s->carry + i; e.episode = s->episode + i;
  e.done_prev = s->done_prev + i;
  e.calls = s->calls + i;
  e.obst = s->obst + (size_t)16 * i;
  return e;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

/* The mission of an env's current episode (the state component of   */
/* Sec. 3.2.1): GoToDoor's target door colour, 0xFF for the families   */
/* without one.                                                        */
static uint8_t mission_of(int family, const uint8_t *obst) {
  return family == FAM_GOTODOOR ? obst[0] : (uint8_t)0xFF;
}

/* Reset every env to episode 0 (reset(key) of Sec. 3.2.2). */
int ox_reset(const ox_batch *b, const ox_state *s, uint8_t *obs, float *reward,
             uint8_t *flags, uint8_t *action, uint8_t *mission, int nthreads) {
  for (int i = 0; i < b->n; ++i)
    if (!ox_side_ok(b->family[i], b->side[i], PARAM(b, i))) return -1;
  if (obs && b->obs_mode >= 4 && !b->sprites) return -1;
  set_threads(nthreads);
  const size_t row_bytes = obs_row_bytes(b);
#pragma omp parallel for schedule(dynamic, 64) if (nthreads > 0)
  for (int i = 0; i < b->n; ++i) {
    ox_env_ref e = env_ref(b, s, i);
    *e.episode = 0;
    ox_layout(b->family[i], b->side[i], PARAM(b, i), b->seed[i], b->rng_id[i],
              0, e.grid, e.x, e.y, e.dir, e.obst);
    *e.t = 0;
    *e.carry = O_EMPTY;
    *e.done_prev = 0;
    *e.calls = 0;
    if (obs)
      emit_obs(b->obs_mode, b->sprites, e.grid, b->side[i], *e.x, *e.y, *e.dir, *e.carry,
               obs_at(b, obs, row_bytes, 0, i));
    if (reward) reward[i] = 0.0f;
    if (flags) flags[i] = OX_FLAG_FIRST;
    if (action) action[i] = OX_ACTION_NONE;
    if (mission) mission[i] = mission_of(b->family[i], e.obst);
  }
  return 0;
}

/* n_steps steps.  actions: [n_steps][N] bytes, or NULL for the random
 * policy (drawn at each env's own call count).  Step k writes output row
 * k % rows. */
int ox_rollout(const ox_batch *b, const ox_state *s, int32_t n_steps,
               const uint8_t *actions, int32_t rows, uint8_t *obs,
               float *reward, uint8_t *flags, uint8_t *action, uint8_t *mission,
               int nthreads) {
  if (rows <= 0 || (obs && b->obs_mode >= 4 && !b->sprites)) return -1;
  set_threads(nthreads);
  const size_t N = (size_t)b->n;
  const size_t row_bytes = obs_row_bytes(b);
#pragma omp parallel for schedule(dynamic, 64) if (nthreads > 0)
  for (int i = 0; i < b->n; ++i) {
    ox_env_ref e = env_ref(b, s, i);
    for (int k = 0; k < n_steps; ++k) {
      size_t row = (size_t)(k % rows);
      uint32_t a;
      if (actions) a = actions[(size_t)k * N + i];
      else a = ox_policy_action(b->seed[i], b->rng_id[i], *e.calls);
      step_one(b->family[i], b->side[i], PARAM(b, i), b->max_steps[i],
               b->seed[i], b->rng_id[i], b->reward_mode, b->obs_mode, b->sprites, e, a,
               obs ? obs_at(b, obs, row_bytes, row, i) : NULL,
               reward + row * N + i,
               flags + row * N + i, action + row * N + i);
      if (mission) mission[row * N + i] = mission_of(b->family[i], e.obst);
      *e.calls += 1u;
    }
  }
  return 0;
}
