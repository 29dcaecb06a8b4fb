// eco_device.h -- device-side definitions shared by the gfx950 kernels of libeco.
//
// Data layout in HBM (all worlds of one object concatenated):
//   per slot (SoA, global slot = world.slot_off + local slot):
//     pos i32, energy i32, age i32, tgt i32 (move / birth target cell),
//     facing u8, flags u8 (bit0 alive, bit1 birth claim made, bit2 birth won),
//     act u8 (action applied), sampled u8 (policy's choice), act_in u8 (injected),
//     uid u64, puid u64, trait f64 (|theta_master|^2)
//   per cell (global cell = world.cell_off + y*W + x):
//     occ i32 (local slot or -1), claim u32 (lowest claiming global slot), res u8, wall u8,
//     sense u8 (the cell's window channels at step start, built before the policy kernel)
//   weights: storage[slot][storage_stride bytes] in the blocked layout below,
//            master[slot][master_stride bytes] FP32 (BF16/FP8 only; FP32 storage is the master)
//   per world: live list segment live[slot_off ..], birth lists, WorldVar, stats ring.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/eco.h"

namespace eco {

constexpr int kStatsRing = 1024;
constexpr uint8_t kAlive = 1, kBirthClaim = 2, kBirthWon = 4;
enum Action : uint8_t { REST = 0, TURN_L = 1, TURN_R = 2, FORWARD = 3, EAT = 4, REPRODUCE = 5, ATTACK = 6 };
// The ecology's eight actions: EAT (4) takes energy, then water, biomass, reproduce;
// with attacks a ninth, attack.
enum EcologyAction : uint8_t { EAT_WATER = 5, EAT_BIOMASS = 6, REPRODUCE_ECO = 7, ATTACK_ECO = 8 };
// Philox stream tags (third counter word).
enum Stream : uint32_t { ST_CELLKEY = 0, ST_FACING = 1, ST_RESINIT = 2, ST_WINIT = 3, ST_ACTION = 4,
                         ST_MUTATE = 5, ST_REGROW = 6, ST_COLOUR_INIT = 7, ST_COLOUR_MUTATE = 8, ST_TERRAIN = 9 };

// Immutable per-world parameters (device table, one entry per world).
struct WorldParams {
  uint32_t W, H, cells, cap;
  uint32_t slot_off, cell_off;
  uint32_t key0, key1;
  uint64_t regrow_thr;          // floor(p * 2^32), compared with a 32-bit draw
  uint64_t density_thr;         // floor(rho * 2^32)
  int32_t e_init, e_cost, e_eat, e_repro, e_child;
  float sigma;
  uint32_t n_init;
  uint32_t has_walls;
  uint32_t attack;              // 1: the attack action kills (the "+A" worlds), 0: it does nothing
  uint32_t pad;
};

// Mutable per-world scalars.
struct WorldVar {
  uint64_t step;
  uint64_t uid_next;
  uint32_t n_live;      // live agents (the live list of this step)
  uint32_t n_births;    // successful births of this step
  uint32_t n_win;       // birth-claim winners of this step
  uint32_t pad;
};

// Counters accumulated by the kernels of one step (u64 atomics), finalised
// into the eco_stats ring by the compaction kernel.
struct StepCounters {
  unsigned long long births, deaths, eaten, regrown, moves_ok, moves_blocked, births_blocked_cell,
      births_blocked_capacity, resource_total;
};

// Weight layouts.  VPL = values per 16-byte block (FP32 4, BF16 8, FP8 16).
// Master (FP32, and FP32 storage):  L1 [KB1][H1][4] | b1[H1] | L2 [H1/4][H2][4] | b2[H2] |
//                                   L3 [R3][H2] | b3[R3]   (rows a >= A of L3/b3 are zero)
// BF16 storage: L1 [ceil(KB1/2)][H1][8] | b1[H1] | L2 [H1/8][H2][8] | b2[H2] | L3 [R3][H2] | b3[R3]
// FP8 storage:  L1 [ceil(KB1/4)][H1][16] | L2 [H1/16][H2][16] | L3 [R3][H2] (bytes) |
//               b1,b2,b3 FP32 | sc1[H1], sc2[H2], sc3[R3] FP32 per-row scales
// R3 = 8 output rows, or 16 with a ninth row: a ninth action, or the log temperature
// after eight (rows and bias slots beyond the head and the temperature are zero).
// KB1 = D/4 (D = 4 S^2 + n_s is a multiple of 4).
struct Layout {
  uint32_t D, S, R, ns, H1, H2, A, wdtype;
  uint32_t ahead0;              // cells ahead of window row 0: R ("Around") or S - 1 ("Front")
  uint32_t temp;                // 1: log temperature stored after the output biases (b3[A])
  uint32_t colour;              // 1: colour trait and rendered colour window
  uint32_t ecology;             // 1: three-resource ecology (cell words of water / energy / biomass levels)
  uint32_t R3;                  // output rows in the weight blocks: 8, or 16 when A + temp > 8
  uint32_t P;                   // logical parameters (the log temperature included)
  uint32_t KB1;                 // FP32 16-byte blocks per L1 row
  uint32_t KBv;                 // storage 16-byte blocks per L1 row
  uint32_t Dpad;                // KBv * VPL (observation buffer length)
  // logical offsets (nn.Linear order)
  uint32_t p_w1, p_b1, p_w2, p_b2, p_w3, p_b3;
  // master unit ranges (a unit = 4 consecutive logical parameters = 16 bytes)
  uint32_t u_w1, u_b1, u_w2, u_b2, u_w3, u_b3, u_end;
  // storage byte offsets
  uint32_t s_w1, s_b1, s_w2, s_b2, s_w3, s_b3, s_sc1, s_sc2, s_sc3;
  uint64_t sstride;             // storage bytes per slot (multiple of 256)
  uint64_t mstride;             // master bytes per slot (0 when storage is FP32)
};

// Pointers of one object's device state.
struct Dev {
  const WorldParams* wp;
  WorldVar* wv;
  StepCounters* cnt;
  eco_stats* ring;              // [n_worlds][kStatsRing]
  int32_t *pos, *energy, *age, *tgt;
  uint8_t *facing, *flags, *act, *sampled, *act_in;
  unsigned long long *uid, *puid;
  double* trait;
  int32_t* occ;
  uint32_t* claim;
  uint32_t* mark;               // [total_cells] step + 1 of the last attack that struck the cell (the
                                // ecology: strikes on the cell this step, cleared by the regrowth
                                // tiles), or null when no world of the object has attacks
  uint8_t *res, *wall;
  uint8_t* sense;               // [total_cells] bit0 agent, bit1 resource, bit2 wall, bits3..5 energy bin
  uint32_t* rgb;                // [total_cells] window words, colour vision: R | G << 8 | B << 16, ecology:
                                // water | energy << 8 | biomass << 16 (levels capped at 255); both with the
                                // agent / resource / wall bits << 24 and, with terrain, the rock height << 27
  const eco_ecology* ep;        // [n_worlds] ecology parameters (null without the ecology)
  int32_t *water, *biomass, *hp;        // [total_slots] ecology: stomach water and biomass, health
  int32_t *cw, *ce, *cb;                // [total_cells] ecology: water, energy, biomass on the grid
  int32_t* rock;                        // [total_cells] terrain: heights 0..31 (null without terrain)
  int8_t* flowdir;                      // [total_cells] terrain: direction the water leaves by, -1 = stays
  int32_t* cw_next;                     // [total_cells] terrain: the water after this step's flow
  float4* colour;               // [total_slots] colour vision only: the colour trait (x, y, z = R, G, B)
  uint8_t* store;               // [total_slots][sstride]
  uint8_t* master;              // [total_slots][mstride] or == store for FP32
  int32_t* live;                // [total_slots], per-world segments at slot_off
  int32_t* bparent;             // [total_slots] birth winners (local slots) by rank
  int32_t* freel;               // [total_slots] free slots (local) ascending
  float* logits;                // [total_slots][lgs]
  uint32_t lgs;                 // logits per slot in that buffer: 8, or 16 with a ninth action
  const double2* trig;          // [256] cos, sin of 2 pi a / 256 (the Box-Muller angle table)
  unsigned long long* cellkeys; // init scratch: [total_cells] (key << 32 | local cell)
  unsigned long long* sorted;   // init scratch
  uint32_t n_worlds;
  uint32_t total_slots;
  uint32_t total_cells;
  uint32_t keep_logits;
  uint32_t inject;
  uint32_t dry;                 // forward only: write sampled/logits, leave the world untouched
};

// Tile of one world's slot or cell range, for per-slot / per-cell kernels.
struct Tile {
  uint32_t world, start, count, pad;
};

// Per-tile scratch of the multi-block passes (slot tiles of 256 slots, cell
// tiles of 1024 cells; a world's tiles are contiguous: tile_rng[4w..4w+3] =
// first/last slot tile, first/last cell tile).
struct TileScratch {
  const Tile* slot_tiles;
  const Tile* cell_tiles;
  const uint32_t* tile_rng;
  uint32_t n_slot_tiles, n_cell_tiles;
  uint32_t* part_slot;   // [slot tiles][16] step counters (actions, moves, meals, deaths, blocked births)
  unsigned long long* part_cell;   // [cell tiles][4] regrown, resource total (ecology: energy), water, biomass
  uint32_t* scan;        // [slot tiles][4] claims, winners, free slots, live slots
  long long* esum;       // [slot tiles] energy sum of live slots
  unsigned long long* ecosum;  // [slot tiles][3] ecology: water, biomass, health of live slots
  double* tmean;         // [slot tiles] mean of the live slots' traits
  double* tm2;           // [slot tiles] sum of squared deviations from that mean
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds, two 32x32->64
// multiplies per round, key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 32x32 -> 64-bit product in one multiply-add instruction (both halves)
    const uint64_t m0 = (uint64_t)0xD2511F53u * c0, m1 = (uint64_t)0xCD9E8D57u * c2;
    // three-input XOR in one instruction (gfx950 bitop3, truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(m1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(m0 >> 32), c3, k1, 0x96);
    c0 = n0;
    c1 = (uint32_t)m1;
    c2 = n2;
    c3 = (uint32_t)m0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

template <typename WP>   // WorldParams, or any struct with the world's key0 / key1
__device__ __forceinline__ uint32_t draw32(const WP& w, uint32_t a, uint32_t step, uint32_t stream) {
  return philox10(a, step, stream, 0u, w.key0, w.key1).x;
}

// Standard normals by the Box-Muller transform (Box & Muller 1958):
// z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2), evaluated in FP64, so that a
// mutated FP32 parameter is the correctly rounded parent + sigma z up to the
// last bits of the FP64 evaluation.  u1 and u2 are 24-bit dyadic fractions,
// which the two functions below use: the logarithm of an integer times a power
// of two, and the angle split at a table of 256 exact multiples of 2 pi / 256.
// ln(m 2^-24) for an integer 1 <= m <= 2^24, in FP64 to about an ulp: m = 2^e f
// with f in [sqrt(1/2), sqrt(2)], so ln(m 2^-24) = (e - 24) ln 2 + ln f with
// ln f = 2 atanh(s), s = (f - 1) / (f + 1), |s| <= 0.1716, from the odd series
// 2 (s + s^3/3 + ... + s^19/19), whose next term is below 2^-55 relative; ln 2
// in two parts, the first with trailing zeros so that (e - 24) times it is exact.
__device__ __forceinline__ double ln_u24(uint32_t m) {
  int e = 31 - __builtin_clz(m);
  double f = ldexp((double)m, -e);   // exact, in [1, 2)
  if (f > 1.4142135623730951) {
    f *= 0.5;
    ++e;
  }
  // s = (f - 1) / (f + 1) (both exact; the divisor lies in [1.7, 2.5]): the
  // hardware reciprocal refined by two Newton steps, then one correction of the
  // quotient by its residual
  const double num = f - 1.0, den = f + 1.0;
  double rc = __builtin_amdgcn_rcp(den);
  rc = __builtin_fma(rc, __builtin_fma(-den, rc, 1.0), rc);
  rc = __builtin_fma(rc, __builtin_fma(-den, rc, 1.0), rc);
  double s = num * rc;
  s = __builtin_fma(rc, __builtin_fma(-den, s, num), s);
  const double s2 = s * s;
  double q = 1.0 / 19.0;
  q = __builtin_fma(q, s2, 1.0 / 17.0);
  q = __builtin_fma(q, s2, 1.0 / 15.0);
  q = __builtin_fma(q, s2, 1.0 / 13.0);
  q = __builtin_fma(q, s2, 1.0 / 11.0);
  q = __builtin_fma(q, s2, 1.0 / 9.0);
  q = __builtin_fma(q, s2, 1.0 / 7.0);
  q = __builtin_fma(q, s2, 1.0 / 5.0);
  q = __builtin_fma(q, s2, 1.0 / 3.0);
  const double two_s = 2.0 * s;
  const double lnf = __builtin_fma(two_s * s2, q, two_s);
  const double k = (double)(e - 24);
  constexpr double ln2_hi = 0x1.62e42fefa38p-1, ln2_lo = 0x1.ef35793c7673p-45;
  return __builtin_fma(k, ln2_hi, __builtin_fma(k, ln2_lo, lnf));
}

// cos and sin of 2 pi j 2^-24 for a 24-bit integer j, in FP64 to a few ulps of
// the value itself: j = 2^16 a + b with a the nearest multiple (b in [-2^15,
// 2^15)), the angle is 2 pi a / 256 (cos, sin from the 256-entry table `tab`)
// plus phi = 2 pi b 2^-24, |phi| <= pi / 256, whose cos and sin come from their
// Taylor series (the first omitted terms, phi^8 / 8! and phi^9 / 9!, are below
// 2^-64), joined by the angle-sum formulas.  The zeros of cos and sin, at the
// quarter turns, are table points with an exact 0 and 1, so next to them the
// result is +-sin phi or +-cos phi and keeps its relative accuracy.
constexpr int kTrigTable = 256;

__device__ __forceinline__ void cossin_2pi_u24(uint32_t j, const double2* __restrict__ tab, double& c, double& s) {
  const uint32_t a = (j + 0x8000u) >> 16;                               // 0..256
  const double2 t = tab[a & (kTrigTable - 1)];
  const double phi = (double)((int)j - (int)(a << 16)) * 0x1.921fb54442d18p-22;   // 2 pi 2^-24
  const double p2 = phi * phi;
  double sp = __builtin_fma(p2, -1.0 / 5040.0, 1.0 / 120.0);
  sp = __builtin_fma(p2, sp, -1.0 / 6.0);
  sp = __builtin_fma(phi * p2, sp, phi);                         // sin phi
  double cp = __builtin_fma(p2, -1.0 / 720.0, 1.0 / 24.0);
  cp = __builtin_fma(p2, cp, -0.5);
  cp = __builtin_fma(p2, cp, 1.0);                               // cos phi
  c = __builtin_fma(t.x, cp, -t.y * sp);
  s = __builtin_fma(t.y, cp, t.x * sp);
}

// sqrt(y) for 0 <= y < 2^10 in FP64, to about an ulp: Goldschmidt's iteration
// (g -> sqrt(y), h -> 1 / (2 sqrt(y))) from the hardware reciprocal square root,
// twice, then one correction by the residual y - g^2.  y = 0 gives 0.
__device__ __forceinline__ double sqrt_small(double y) {
  const double r0 = __builtin_amdgcn_rsq(y);
  double g = y * r0, h = 0.5 * r0;
  double e = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, e, g);
  h = __builtin_fma(h, e, h);
  e = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, e, g);
  h = __builtin_fma(h, e, h);
  g = __builtin_fma(__builtin_fma(-g, g, y), h, g);
  return y > 0.0 ? g : 0.0;
}

// Four standard normals from one Philox block (tab: the angle table above, in LDS).
__device__ __forceinline__ void gauss4k(uint32_t key0, uint32_t key1, uint32_t a, uint32_t step, uint32_t stream,
                                        uint32_t blk, const double2* __restrict__ tab, double z[4]) {
  const uint4 x = philox10(a, step, stream, blk, key0, key1);
  const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double r = sqrt_small(-2.0 * ln_u24((xs[2 * p] >> 8) + 1u));   // u1 = ((x >> 8) + 1) 2^-24
    double s, c;
    cossin_2pi_u24(xs[2 * p + 1] >> 8, tab, c, s);                 // u2 = (x >> 8) 2^-24
    z[2 * p] = r * c;
    z[2 * p + 1] = r * s;
  }
}

__device__ __forceinline__ void gauss4(const WorldParams& w, uint32_t a, uint32_t step, uint32_t stream,
                                       uint32_t blk, const double2* __restrict__ tab, double z[4]) {
  gauss4k(w.key0, w.key1, a, step, stream, blk, tab, z);
}

// The angle table into LDS (all threads of the block take part).
__device__ __forceinline__ void load_trig(const double2* __restrict__ src, double2* dst) {
  for (int i = threadIdx.x; i < kTrigTable; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
}

__device__ __forceinline__ int dir_dx(int f) { return f == 1 ? 1 : (f == 3 ? -1 : 0); }
__device__ __forceinline__ int dir_dy(int f) { return f == 0 ? -1 : (f == 2 ? 1 : 0); }

// Local cell one step from `cell` along facing f (sign = +1 ahead, -1 behind), torus.
template <typename WP>   // WorldParams, or any struct with the world's W and H
__device__ __forceinline__ uint32_t neighbour(const WP& w, uint32_t cell, int f, int sign) {
  int x = (int)(cell % w.W), y = (int)(cell / w.W);
  x += sign * dir_dx(f);
  y += sign * dir_dy(f);
  if (x < 0) x += (int)w.W; else if (x >= (int)w.W) x -= (int)w.W;
  if (y < 0) y += (int)w.H; else if (y >= (int)w.H) y -= (int)w.H;
  return (uint32_t)y * w.W + (uint32_t)x;
}

// Local cell `ahead` steps along facing f and `side` steps to the right of that
// heading (negative: to the left), torus; |ahead|, |side| <= 3.  Used for the
// attack square, so not on the hot path of the step.
template <typename WP>
__device__ __forceinline__ uint32_t offset_cell(const WP& w, uint32_t cell, int f, int ahead, int side) {
  const int r = (f + 1) & 3;
  int x = (int)(cell % w.W) + ahead * dir_dx(f) + side * dir_dx(r);
  int y = (int)(cell / w.W) + ahead * dir_dy(f) + side * dir_dy(r);
  x %= (int)w.W;
  y %= (int)w.H;
  if (x < 0) x += (int)w.W;
  if (y < 0) y += (int)w.H;
  return (uint32_t)y * w.W + (uint32_t)x;
}

// Wave-local LDS ordering: keeps the compiler from moving LDS accesses across
// this point; LDS operations of one wave complete in issue order.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Index of the world whose [off[w], off[w+1]) range holds g (off in LDS, n worlds).
__device__ __forceinline__ uint32_t find_world(const uint32_t* off, uint32_t n, uint32_t g) {
  uint32_t lo = 0, hi = n;  // off[lo] <= g < off[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace eco
