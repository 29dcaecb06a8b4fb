// eco_step.hip -- world-dynamics kernels of one step, and the init kernels.
//
// Step order (the policy kernel in eco_forward.hip runs first and has already
// applied turns and made the forward-move claims on the pre-step occupancy):
//   k_move         winners move; EAT; step cost; death at energy <= 0; age
//                  (Sec. 3.2 "Resources and Agent Health", "Actions")
//   k_birth_claim  eligible parents claim the empty cell behind them
//                  (Sec. 3.2 "Actions": child placed directly behind the parent)
//   k_birth_scan   per world: winners ranked in slot order, free slots listed in
//                  ascending order (the recycled-slot free list)
//   k_birth_commit child state + child weights = parent + sigma * N(0,1)
//                  (Sec. 3.3 mutation) into the recycled slot
//   k_regrow       each empty cell regrows one unit with probability p
//                  (Sec. 3.2: energy slowly grows back)
//   k_compact      per world: live list of the next step and the step's
//                  statistics (App. E measurement interface)
// Every contended write is an atomicMin on a claim word; every other write goes
// to a unique slot or cell, so the integer state is independent of scheduling.
#include <mutex>

#include "eco_device.h"

namespace eco {

constexpr int kSlotTile = 256;   // slots per block in per-slot kernels
// Cell tiles (1024 cells each) are built on the host; per-cell kernels take one tile per block.
constexpr int kScanThreads = 1024;
constexpr int kSlotPart = 16;    // u32 counters per slot tile
constexpr int kCellPart = 4;     // u64 counters per cell tile

// Per-slot-tile counters (index in the partials row).
enum { PC_HIST = 0, PC_MOVES_OK = 9, PC_MOVES_BLOCKED = 10, PC_EATEN = 11, PC_DEATHS = 12, PC_BB_CELL = 13,
       PC_KILLED = 14 };

// ---------------------------------------------------------------------------
// Small block helpers
// ---------------------------------------------------------------------------
// Wave-wide sums by DPP, the data-parallel lane moves of the VALU: lane i of
// each row of 16 lanes adds row lanes i - 1, i - 2, i - 4, i - 8 (taking 0 past
// the row's start), then rows 1 and 3 add the last lane of rows 0 and 2, and
// rows 2 and 3 the last lane of row 1.  Each step is a few VALU cycles where a
// lane shuffle goes through the LDS crossbar.  Every lane of the wave must be
// active.  64-bit values move as two 32-bit halves.
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_move(T x) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(
        T, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)__builtin_bit_cast(uint32_t, x), CTRL, ROWS, 0xf, false));
  } else {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xf, false);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

// Inclusive sum over lanes 0..lane of the wave (a fixed order for FP64).
template <typename T>
__device__ __forceinline__ T wave_scan(T x) {
  x += dpp_move<0x111, 0xf>(x);   // row_shr:1
  x += dpp_move<0x112, 0xf>(x);   // row_shr:2
  x += dpp_move<0x114, 0xf>(x);   // row_shr:4
  x += dpp_move<0x118, 0xf>(x);   // row_shr:8
  x += dpp_move<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
  x += dpp_move<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
  return x;
}

// x of lane l (the same l in every lane).
template <typename T>
__device__ __forceinline__ T lane_value(T x, int l) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, (uint32_t)__builtin_amdgcn_readlane((int)__builtin_bit_cast(uint32_t, x), l));
  } else {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

template <int NT>
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_scan(v);
  if (lane == 63) red[wave] = v;
  __syncthreads();
  unsigned long long t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) t += red[i];
  __syncthreads();
  return t;  // valid in thread 0
}

// Deterministic FP64 block sum: a fixed order within each wave, then waves in order.
template <int NT>
__device__ __forceinline__ double block_sum_f64(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_scan(v);
  if (lane == 63) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) t += red[i];
  __syncthreads();
  return t;  // valid in thread 0
}

// Exclusive scan of one u32 per thread over the block; returns the exclusive
// prefix, *total gets the block total (all threads).
template <int NT>
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t* red, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_scan(v);
  if (lane == 63) red[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int i = 0; i < NT / 64; ++i) {
      const uint32_t t = red[i];
      red[i] = run;
      run += t;
    }
    red[NT / 64] = run;
  }
  __syncthreads();
  const uint32_t ex = red[wave] + inc - v;
  *total = red[NT / 64];
  __syncthreads();
  return ex;
}

// Sum of the per-wave values r_i (lane i of every wave holding r_i, i < NW,
// zero in the other lanes) over the waves before the calling one; *all gets the
// sum over all NW waves.  Every wave computes both the same way.
template <int NW, typename T>
__device__ __forceinline__ T waves_before(T r, T* all) {
  static_assert(NW >= 1 && NW <= 64, "at most 64 waves");
  const int wave = threadIdx.x >> 6;
  r = wave_scan(r);
  *all = lane_value(r, NW - 1);
  const T b = lane_value(r, wave > 0 ? wave - 1 : 0);
  return wave > 0 ? b : T(0);
}

// Exclusive scan of one u64 per thread over the block with one barrier: each
// wave reads the waves' totals from red itself.  red[NT / 64] must not be
// written again before every thread has returned (the caller's next barrier).
template <int NT>
__device__ __forceinline__ unsigned long long block_exscan_u64(unsigned long long v, unsigned long long* red,
                                                             unsigned long long* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long inc = wave_scan(v);
  if (lane == 63) red[wave] = inc;
  __syncthreads();
  const unsigned long long before = waves_before<NT / 64>(lane < NT / 64 ? red[lane] : 0ull, total);
  return before + inc - v;
}

// Block counters in LDS with one atomic per wave instead of one per lane (the
// atomics of a wave's lanes on one LDS address run one after another, several
// cycles each).  count_lanes: adds the number of the wave's active lanes to *c
// (called in the branch whose lanes are counted).  count_lanes_by<N>: adds, for
// each k < N, the number of active lanes whose v is k to c[k].  wave_add_u64:
// adds the sum of v over the wave to *c (every lane of the wave active).
__device__ __forceinline__ void count_lanes(uint32_t* c) {
  const uint64_t m = __ballot(1);
  if ((threadIdx.x & 63u) == (uint32_t)__builtin_ctzll(m)) atomicAdd(c, (uint32_t)__builtin_popcountll(m));
}

template <int N>
__device__ __forceinline__ void count_lanes_by(uint32_t* c, int v) {
  const uint32_t first = (uint32_t)__builtin_ctzll(__ballot(1));
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const uint64_t m = __ballot(v == k);
    if (m && (threadIdx.x & 63u) == first) atomicAdd(&c[k], (uint32_t)__builtin_popcountll(m));
  }
}

__device__ __forceinline__ void wave_add_u64(unsigned long long v, unsigned long long* c) {
  v = wave_scan(v);
  if ((threadIdx.x & 63u) == 63 && v) atomicAdd(c, v);
}

// ---------------------------------------------------------------------------
// Weight emission (init, mutation, re-quantisation) for one agent, one block.
// A "unit" is 4 consecutive logical parameters = one 16-byte FP32 master block.
// ---------------------------------------------------------------------------
struct UnitInfo {
  uint32_t p;      // logical index of the first parameter
  uint32_t nvalid; // parameters of the unit that exist (0..4)
  int layer;       // 0,1,2 weights; 3,4,5 biases of layer 0,1,2
  uint32_t row;    // output row (weights) / first row (biases)
  uint32_t kb;     // k-block (weights of layers 0,1) or column quad (layer 2)
};

__device__ __forceinline__ UnitInfo unit_info(const Layout& L, uint32_t u) {
  UnitInfo r;
  if (u < L.u_b1) {                 // W1 [kb][j]
    r.layer = 0; r.kb = u / L.H1; r.row = u % L.H1;
    r.p = L.p_w1 + r.row * L.D + 4 * r.kb; r.nvalid = 4;
  } else if (u < L.u_w2) {          // b1
    r.layer = 3; r.row = 4 * (u - L.u_b1); r.kb = 0;
    r.p = L.p_b1 + r.row; r.nvalid = 4;
  } else if (u < L.u_b2) {          // W2 [kb][i]
    const uint32_t e = u - L.u_w2;
    r.layer = 1; r.kb = e / L.H2; r.row = e % L.H2;
    r.p = L.p_w2 + r.row * L.H1 + 4 * r.kb; r.nvalid = 4;
  } else if (u < L.u_w3) {          // b2
    r.layer = 4; r.row = 4 * (u - L.u_b2); r.kb = 0;
    r.p = L.p_b2 + r.row; r.nvalid = 4;
  } else if (u < L.u_b3) {          // W3 [a][H2], 4 columns per unit
    const uint32_t e = u - L.u_w3, per = L.H2 / 4;
    r.layer = 2; r.row = e / per; r.kb = e % per;
    r.p = L.p_w3 + r.row * L.H2 + 4 * r.kb; r.nvalid = (r.row < L.A) ? 4 : 0;
  } else {                          // b3 (R3 padded), then the log temperature in slot A when it evolves
    const uint32_t e = u - L.u_b3, n3 = L.A + L.temp;
    r.layer = 5; r.row = 4 * e; r.kb = 0;
    r.p = L.p_b3 + r.row;
    r.nvalid = (r.row < n3) ? min(4u, n3 - r.row) : 0;
  }
  return r;
}

// Round-to-nearest-even FP32 -> BF16 of a finite value.
__device__ __forceinline__ uint32_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// FP32 -> OCP FP8 E4M3FN, round to nearest even, saturating at 448; values
// that round to zero give +0.  Works on the magnitude's bit pattern: the
// E4M3 exponent range is [-6, 8], subnormal step 2^-9.
__device__ __forceinline__ uint32_t fp8_rne_sat(float x) {
  const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fabsf(x);
  if (!(a < 448.0f)) return sign | 0x7Eu;
  uint32_t q;
  if (a < 0x1p-6f) {
    // subnormal range: q = RNE(a / 2^-9) in 0..8 (8 = smallest normal, code 0x08)
    const float t = a * 512.0f;        // exact (power-of-two scale)
    q = (uint32_t)__builtin_rintf(t);  // round half to even
  } else {
    const uint32_t u = __float_as_uint(a);
    const int e = (int)(u >> 23) - 127;               // -6 .. 8
    const uint32_t mant = u & 0x7FFFFFu;
    uint32_t m3 = mant >> 20;                         // top 3 mantissa bits
    const uint32_t rest = mant & 0xFFFFFu;            // 20 dropped bits
    const uint32_t half = 0x80000u;
    if (rest > half || (rest == half && (m3 & 1u))) ++m3;
    uint32_t ee = (uint32_t)(e + 7);
    if (m3 == 8) { m3 = 0; ++ee; }
    q = (ee << 3) | m3;
    if (q > 0x7Eu) q = 0x7Eu;
  }
  if (q == 0) return 0u;
  return sign | q;
}

__device__ __forceinline__ float fp8_value(uint32_t q) {
  const uint32_t e = (q >> 3) & 15u, m = q & 7u;
  float v = (e == 0) ? (float)m * 0x1p-9f : ldexpf(1.0f + (float)m * 0.125f, (int)e - 7);
  return (q & 0x80u) ? -v : v;
}

enum EmitMode { EMIT_INIT = 0, EMIT_REQUANT = 2 };

// Writes the FP32 master of global slot `child` and its storage copy, and the
// trait |theta|^2 (init and weight writes; births go through mutate_child).
// INIT: N(0, 1/fan_in) weights from (rng_slot, step 0, WINIT), zero biases.
// REQUANT: master already written.
template <int WDT>
__device__ void emit_agent(const Dev& d, const Layout& L, const WorldParams& wp, uint32_t child, int mode,
                           uint32_t rng_slot, double std1, double std2, double std3, const double2* tab,
                           uint32_t* s_amax, double* s_red) {
  const int tid = threadIdx.x;
  float* mc = reinterpret_cast<float*>(d.master + (uint64_t)child * L.mstride);
  uint8_t* sc = d.store + (uint64_t)child * L.sstride;
  const uint32_t nrows = L.H1 + L.H2 + L.R3;
  if (WDT == 2) {
    for (uint32_t i = tid; i < nrows; i += blockDim.x) s_amax[i] = 0u;
    __syncthreads();
  }
  if (L.colour && tid == 0 && mode == EMIT_INIT) {
    // colour trait: U[0,1) per channel
    const uint4 x = philox10(rng_slot, 0u, ST_COLOUR_INIT, 0u, wp.key0, wp.key1);
    d.colour[child] = make_float4((float)(x.x >> 8) * 0x1p-24f, (float)(x.y >> 8) * 0x1p-24f,
                                  (float)(x.z >> 8) * 0x1p-24f, 0.0f);
  }
  double tsum = 0.0;
  for (uint32_t u = tid; u < L.u_end; u += blockDim.x) {
    const UnitInfo ui = unit_info(L, u);
    float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (mode == EMIT_REQUANT) {
      const float4 m4 = reinterpret_cast<const float4*>(mc)[u];
      v[0] = m4.x; v[1] = m4.y; v[2] = m4.z; v[3] = m4.w;
    } else if (ui.nvalid > 0 && ui.layer < 3) {
      double z[4];
      gauss4(wp, rng_slot, 0u, ST_WINIT, ui.p >> 2, tab, z);
      const double sd = ui.layer == 0 ? std1 : (ui.layer == 1 ? std2 : std3);
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = (float)(z[i] * sd);
    }
    if (mode != EMIT_REQUANT) reinterpret_cast<float4*>(mc)[u] = make_float4(v[0], v[1], v[2], v[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) tsum += (double)v[i] * (double)v[i];

    if (WDT == 1) {
      const uint32_t lo = bf16_rne(v[0]) | (bf16_rne(v[1]) << 16);
      const uint32_t hi = bf16_rne(v[2]) | (bf16_rne(v[3]) << 16);
      uint64_t off;
      if (ui.layer == 0) off = L.s_w1 + ((uint64_t)(ui.kb >> 1) * L.H1 + ui.row) * 16 + (ui.kb & 1) * 8;
      else if (ui.layer == 1) off = L.s_w2 + ((uint64_t)(ui.kb >> 1) * L.H2 + ui.row) * 16 + (ui.kb & 1) * 8;
      else if (ui.layer == 2) off = L.s_w3 + ((uint64_t)ui.row * L.H2 + 4 * ui.kb) * 2;
      else if (ui.layer == 3) off = L.s_b1 + (uint64_t)ui.row * 2;
      else if (ui.layer == 4) off = L.s_b2 + (uint64_t)ui.row * 2;
      else off = L.s_b3 + (uint64_t)ui.row * 2;
      *reinterpret_cast<uint2*>(sc + off) = make_uint2(lo, hi);
    } else if (WDT == 2) {
      if (ui.layer < 3) {
        const uint32_t r = ui.layer == 0 ? ui.row : (ui.layer == 1 ? L.H1 + ui.row : L.H1 + L.H2 + ui.row);
        float mx = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) mx = fmaxf(mx, fabsf(v[i]));
        atomicMax(&s_amax[r], __float_as_uint(mx));
      } else {
        const uint64_t off = (ui.layer == 3 ? L.s_b1 : (ui.layer == 4 ? L.s_b2 : L.s_b3)) + (uint64_t)ui.row * 4;
        *reinterpret_cast<float4*>(sc + off) = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  }
  if (WDT == 2) {
    __syncthreads();
    // scales, then a second pass over the same units (each thread re-reads its own writes)
    for (uint32_t r = tid; r < nrows; r += blockDim.x) {
      const float amax = __uint_as_float(s_amax[r]);
      const float scale = amax > 0.0f ? amax / 448.0f : 1.0f;
      uint64_t off;
      if (r < L.H1) off = L.s_sc1 + (uint64_t)r * 4;
      else if (r < L.H1 + L.H2) off = L.s_sc2 + (uint64_t)(r - L.H1) * 4;
      else off = L.s_sc3 + (uint64_t)(r - L.H1 - L.H2) * 4;
      *reinterpret_cast<float*>(sc + off) = scale;
    }
    for (uint32_t u = tid; u < L.u_end; u += blockDim.x) {
      const UnitInfo ui = unit_info(L, u);
      if (ui.layer >= 3) continue;
      const uint32_t r = ui.layer == 0 ? ui.row : (ui.layer == 1 ? L.H1 + ui.row : L.H1 + L.H2 + ui.row);
      const float amax = __uint_as_float(s_amax[r]);
      const float scale = amax > 0.0f ? amax / 448.0f : 1.0f;
      const float4 m4 = reinterpret_cast<const float4*>(mc)[u];
      const uint32_t q = fp8_rne_sat(m4.x / scale) | (fp8_rne_sat(m4.y / scale) << 8) |
                         (fp8_rne_sat(m4.z / scale) << 16) | (fp8_rne_sat(m4.w / scale) << 24);
      uint64_t off;
      if (ui.layer == 0) off = L.s_w1 + ((uint64_t)(ui.kb >> 2) * L.H1 + ui.row) * 16 + (ui.kb & 3) * 4;
      else if (ui.layer == 1) off = L.s_w2 + ((uint64_t)(ui.kb >> 2) * L.H2 + ui.row) * 16 + (ui.kb & 3) * 4;
      else off = L.s_w3 + (uint64_t)ui.row * L.H2 + 4 * ui.kb;
      *reinterpret_cast<uint32_t*>(sc + off) = q;
    }
  }
  const double t = block_sum_f64<256>(tsum, s_red);
  if (tid == 0) d.trait[child] = t;
}

// ---------------------------------------------------------------------------
// Step kernels
// ---------------------------------------------------------------------------
// Winners move, then EAT, step cost, death, age; per-tile counters.
// Three-resource ecology, one live agent after the moves (it touches only its own
// cell c, which no other agent touches in this launch): eat the chosen resource
// (up to the eat amount, the cell's content and the room under the stomach cap);
// pay energy (destroyed; rest costs least) and water (onto the cell); each
// resource that ran short, the agent's age and each of the `hits` strikes on its
// cell this step cost health; at zero health the agent dies and leaves water,
// energy and biomass on its cell (killed, when struck); otherwise energy heals
// it below full health and it ages.  Returns the new energy.
__device__ __forceinline__ int ecology_agent(const Dev& d, const eco_ecology& e, const WorldParams& wp, uint32_t slot,
                                             uint32_t c, int a, uint32_t hits, uint32_t* cnt) {
  int E = d.energy[slot], Wt = d.water[slot], B = d.biomass[slot], hp = d.hp[slot];
  int t = 0;
  if (a == EAT) {
    t = min(min(wp.e_eat, d.ce[c]), e.cap_energy - E);
    if (t > 0) { d.ce[c] -= t; E += t; }
  } else if (a == EAT_WATER) {
    t = min(min(e.eat_water, d.cw[c]), e.cap_water - Wt);
    if (t > 0) { d.cw[c] -= t; Wt += t; }
  } else if (a == EAT_BIOMASS) {
    t = min(min(e.eat_biomass, d.cb[c]), e.cap_biomass - B);
    if (t > 0) { d.cb[c] -= t; B += t; }
  }
  if (t > 0) count_lanes(&cnt[PC_EATEN]);
  int over = 0;
  E -= (a == REST) ? wp.e_cost : e.e_cost_move;
  if (E < 0) { E = 0; ++over; }
  const int spend = min(Wt, e.w_cost);
  Wt -= spend;
  d.cw[c] += spend;
  if (spend < e.w_cost) ++over;
  const long long damage =
      (long long)over * e.hp_overspend + (d.age[slot] >> e.age_shift) + (long long)hits * e.attack_damage;
  if ((long long)hp - damage <= 0) {
    d.cw[c] += Wt;
    d.ce[c] += E;
    d.cb[c] += B;
    E = Wt = B = hp = 0;
    d.flags[slot] = 0;
    d.occ[c] = -1;
    count_lanes(&cnt[PC_DEATHS]);
    if (hits) count_lanes(&cnt[PC_KILLED]);
  } else {
    hp -= (int)damage;
    if (hp < e.hp_max && E >= e.heal_energy) {
      hp = min(hp + e.hp_heal, e.hp_max);
      E -= e.heal_energy;
    }
    d.age[slot] += 1;
  }
  d.water[slot] = Wt;
  d.biomass[slot] = B;
  d.hp[slot] = hp;
  return E;
}

// One live agent's move (a FORWARD winner takes its claimed cell), then EAT, the
// step cost and death (Sec. 3.2), or with the ecology ecology_agent; counts into
// the LDS counters cnt.  stamp: the attack stamp of this step (step + 1).
__device__ __forceinline__ void move_agent(const Dev& d, const WorldParams& wp, uint32_t w, uint32_t slot,
                                           uint32_t local, uint32_t stamp, uint32_t* cnt) {
  // every load the non-ecology rules can need, issued before any store: the
  // agent's fields, then the cells it stands on or claimed (no other agent
  // writes these cells in this pass: a claim targets a cell free at step start)
  const int a = d.act[slot];
  int cell = d.pos[slot];
  const int t = d.tgt[slot];
  int E = d.energy[slot];
  const uint32_t won = (a == FORWARD && t >= 0) ? d.claim[wp.cell_off + t] : ~0u;
  const uint8_t r0 = d.ep ? 0 : d.res[wp.cell_off + cell];
  const uint32_t m0 = (!d.ep && wp.attack) ? d.mark[wp.cell_off + cell] : 0u;
  const uint32_t m1 = (!d.ep && wp.attack && a == FORWARD && t >= 0) ? d.mark[wp.cell_off + t] : 0u;
  count_lanes_by<9>(&cnt[PC_HIST], a);
  bool moved = false;
  if (a == FORWARD) {
    if (t >= 0 && won == slot) {
      d.claim[wp.cell_off + t] = 0xFFFFFFFFu;
      d.occ[wp.cell_off + cell] = -1;
      d.occ[wp.cell_off + t] = (int)local;
      cell = t;
      moved = true;
      d.pos[slot] = cell;
      count_lanes(&cnt[PC_MOVES_OK]);
    } else {
      count_lanes(&cnt[PC_MOVES_BLOCKED]);
    }
  }
  if (d.ep) {
    const uint32_t g = wp.cell_off + (uint32_t)cell;
    E = ecology_agent(d, d.ep[w], wp, slot, g, a, wp.attack ? d.mark[g] : 0u, cnt);
  } else if (wp.attack && (moved ? m1 : m0) == stamp) {
    // struck after the moves: dies where it stands; its carried energy goes
    // back to the cell as one resource unit (cells hold 0 or 1 unit)
    d.flags[slot] = 0;
    d.occ[wp.cell_off + cell] = -1;
    d.res[wp.cell_off + cell] = 1;
    E = 0;
    count_lanes(&cnt[PC_DEATHS]);
    count_lanes(&cnt[PC_KILLED]);
  } else {
    if (a == EAT && r0 > 0) {   // an eater did not move: cell is its own
      d.res[wp.cell_off + cell] = (uint8_t)(r0 - 1);
      E += wp.e_eat;
      count_lanes(&cnt[PC_EATEN]);
    }
    E -= wp.e_cost;
    if (E <= 0) {
      d.flags[slot] = 0;
      d.occ[wp.cell_off + cell] = -1;
      count_lanes(&cnt[PC_DEATHS]);
    } else {
      d.age[slot] += 1;
    }
  }
  d.energy[slot] = E;
}

__global__ __launch_bounds__(kSlotTile) void k_move(Dev d, const Tile* __restrict__ tiles, uint32_t* __restrict__ part) {
  __shared__ uint32_t cnt[kSlotPart];
  if (threadIdx.x < kSlotPart) cnt[threadIdx.x] = 0;
  __syncthreads();
  const Tile tl = tiles[blockIdx.x];
  const WorldParams wp = d.wp[tl.world];
  const uint32_t stamp = (uint32_t)d.wv[tl.world].step + 1u;   // attack stamp of this step
  if (threadIdx.x < tl.count) {
    const uint32_t local = tl.start + threadIdx.x;
    const uint32_t slot = wp.slot_off + local;
    if (d.flags[slot] & kAlive) move_agent(d, wp, tl.world, slot, local, stamp, cnt);
  }
  __syncthreads();
  if (threadIdx.x < kSlotPart && threadIdx.x != PC_BB_CELL)   // the birth claims write PC_BB_CELL
    part[blockIdx.x * kSlotPart + threadIdx.x] = cnt[threadIdx.x];
}

// Eligible parents claim the empty cell directly behind them (slot tiles), and
// in the same launch each cell tile regrows its empty cells (independent work:
// regrowth reads and writes only the resource layer).
// One slot's birth claim: an eligible live parent claims the empty cell directly
// behind it (lowest slot wins, atomicMin); a parent whose cell behind is taken or
// walled counts as blocked.
// Returns whether the slot claimed a cell.
__device__ __forceinline__ bool birth_claim_slot(const Dev& d, const WorldParams& wp, uint32_t w, uint32_t slot,
                                                 uint32_t n_actions, uint32_t* blocked) {
  const uint8_t fl = d.flags[slot];
  if (!(fl & kAlive)) return false;
  bool eligible = d.energy[slot] >= wp.e_repro && (n_actions == 5 || d.act[slot] == REPRODUCE);
  if (d.ep) {   // ecology: the eighth action, and spare biomass and water to give the child
    const eco_ecology& e = d.ep[w];
    eligible = d.act[slot] == REPRODUCE_ECO && d.energy[slot] >= wp.e_repro && d.water[slot] >= e.w_child &&
               d.biomass[slot] >= e.b_repro;
  }
  if (eligible) {
    const uint32_t t = neighbour(wp, (uint32_t)d.pos[slot], d.facing[slot], -1);
    const bool walled = wp.has_walls && d.wall[wp.cell_off + t];
    if (d.occ[wp.cell_off + t] == -1 && !walled) {
      atomicMin(&d.claim[wp.cell_off + t], slot);
      d.tgt[slot] = (int)t;
      d.flags[slot] = fl | kBirthClaim;
      return true;
    }
    count_lanes(blocked);
  }
  return false;
}

__device__ __forceinline__ void birth_claim_tile(const Dev& d, const TileScratch& ts, uint32_t tile, uint32_t n_actions,
                                                 uint32_t* blocked) {
  const Tile tl = ts.slot_tiles[tile];
  const WorldParams wp = d.wp[tl.world];
  if (threadIdx.x < tl.count) birth_claim_slot(d, wp, tl.world, wp.slot_off + tl.start + threadIdx.x, n_actions, blocked);
  __syncthreads();
  if (threadIdx.x == 0) ts.part_slot[tile * kSlotPart + PC_BB_CELL] = *blocked;
}

// floor(min(1, rate * b) * 2^32) in exact integer arithmetic, for a finite rate >= 0
// and b >= 1: rate = M 2^E with an integer M < 2^24, so rate * b * 2^32 is the
// integer M b (< 2^55) scaled by 2^(E + 32), floored.
__device__ __forceinline__ uint64_t photo_threshold(float rate, int b) {
  const uint32_t u = __float_as_uint(rate);
  const uint32_t ex = (u >> 23) & 0xFFu;
  const uint64_t M = ex ? ((u & 0x7FFFFFu) | 0x800000u) : (u & 0x7FFFFFu);
  const int k = (ex ? (int)ex - 150 : -149) + 32;   // rate = M 2^(k - 32)
  const uint64_t mb = M * (uint64_t)(uint32_t)b;
  constexpr uint64_t one = 1ull << 32;
  if (mb == 0) return 0;
  if (k >= 0) return (k >= 32 || mb >= (one >> k)) ? one : (mb << k);
  if (k <= -64) return 0;
  const uint64_t v = mb >> (-k);
  return v > one ? one : v;
}

// The regrowth (and photosynthesis) draws of local cells 4 q .. 4 q + 3 at `step`:
// one Philox block, output j for cell 4 q + j.
__device__ __forceinline__ uint4 regrow_draws(const WorldParams& wp, uint32_t q, uint32_t step) {
  return philox10(q, step, ST_REGROW, 0u, wp.key0, wp.key1);
}

__device__ __forceinline__ uint32_t word_of(const uint4& x, int j) {
  return j == 0 ? x.x : (j == 1 ? x.y : (j == 2 ? x.z : x.w));
}

// One regrowth pass over the resource bytes of local cells c0 .. c0 + n - 1 (c0 a
// multiple of 4, n <= 4) held in the word v: each empty cell regrows one unit
// with probability p (its draw against floor(p 2^32)).  Returns the new word;
// adds the regrown cells and the resource total to grown and total.
__device__ __forceinline__ uint32_t regrow_word(const WorldParams& wp, uint32_t c0, uint32_t n, uint32_t v,
                                                uint32_t step, unsigned long long& grown, unsigned long long& total) {
  bool any = false;
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j) any |= j < n && ((v >> (8 * j)) & 0xFFu) == 0;
  uint32_t nv = v;
  if (any) {
    const uint4 x = regrow_draws(wp, c0 >> 2, step);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
      if (j < n && ((v >> (8 * j)) & 0xFFu) == 0 && (uint64_t)word_of(x, (int)j) < wp.regrow_thr) {
        nv |= 1u << (8 * j);
        ++grown;
      }
  }
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j)
    if (j < n) total += (nv >> (8 * j)) & 0xFFu;
  return nv;
}

// Regrowth of the cells of tile tl (one resource layer), four cells per thread
// and pass (tiles start at multiples of 1024 cells; the cell allocation ends at a
// multiple of 64, so the last word of a tile stays inside it); the regrown count
// and the resource total go to cnt[0], cnt[1] (LDS).
__device__ __forceinline__ void regrow_cells(const Dev& d, const WorldParams& wp, const Tile tl, uint32_t step,
                                             unsigned long long* cnt) {
  unsigned long long grown = 0, total = 0;
  for (uint32_t i = 4 * threadIdx.x; i < tl.count; i += 4 * blockDim.x) {
    const uint32_t c0 = tl.start + i, n = min(4u, tl.count - i);
    uint8_t* rp = d.res + wp.cell_off + c0;
    const uint32_t v = *reinterpret_cast<const uint32_t*>(rp);
    const uint32_t nv = regrow_word(wp, c0, n, v, step, grown, total);
    if (nv != v) {
      if (n == 4) {
        *reinterpret_cast<uint32_t*>(rp) = nv;
      } else {
        for (uint32_t j = 0; j < n; ++j) rp[j] = (uint8_t)(nv >> (8 * j));
      }
    }
  }
  wave_add_u64(grown, &cnt[0]);
  wave_add_u64(total, &cnt[1]);
}

// Four consecutive int32 cells from g (g a multiple of 4; the cell allocation ends
// at a multiple of 64, so the vector stays inside it even for a ragged tail) and
// their store, whole for n = 4, else cell by cell.
__device__ __forceinline__ void load_cells4(const int32_t* p, int v[4]) {
  const int4 x = *reinterpret_cast<const int4*>(p);
  v[0] = x.x;
  v[1] = x.y;
  v[2] = x.z;
  v[3] = x.w;
}

__device__ __forceinline__ void store_cells4(int32_t* p, uint32_t n, const int v[4]) {
  if (n == 4) {
    *reinterpret_cast<int4*>(p) = make_int4(v[0], v[1], v[2], v[3]);
  } else {
    for (uint32_t j = 0; j < n; ++j) p[j] = v[j];
  }
}

__device__ __forceinline__ int byte_of(uint32_t v, int j) { return (int)(int8_t)(uint8_t)(v >> (8 * j)); }

// Terrain: the water on local cells c0 .. c0 + n - 1 after the flow (each cell's
// water moves one cell downhill, every cell at once): a cell keeps its own water if
// it has no way down, and takes that of each neighbour whose way down leads to it.
// own[] holds the cells' water before the flow, fd their four direction bytes.
// With W a multiple of 4 a whole group lies in one row, and the neighbours above
// and below are whole aligned groups: flow_rows_load reads them (and the cells
// left and right of the group) so that the caller can issue these loads with its
// own, and returns false where the group takes the per-cell path instead.
struct FlowRows {
  int wu[4], wd[4];   // water of the cells above and below
  uint32_t fu, fdn;   // their direction bytes
  int wl, wr, fl, fr;   // water and direction of the cells left and right of the group
};

__device__ __forceinline__ bool flow_rows_load(const Dev& d, const WorldParams& wp, uint32_t c0, uint32_t n,
                                               FlowRows& r) {
  if ((wp.W & 3u) != 0 || n != 4) return false;
  const uint32_t off = wp.cell_off, W = wp.W, y0 = c0 / W, x0 = c0 - y0 * W, row = y0 * W;
  const uint32_t up = (y0 == 0 ? wp.H - 1 : y0 - 1) * W + x0, dn = (y0 + 1 == wp.H ? 0u : y0 + 1) * W + x0;
  const uint32_t lf = row + (x0 == 0 ? W - 1 : x0 - 1), rt = row + (x0 + 4 == W ? 0u : x0 + 4);
  load_cells4(d.cw + off + up, r.wu);
  load_cells4(d.cw + off + dn, r.wd);
  r.fu = *reinterpret_cast<const uint32_t*>(d.flowdir + off + up);
  r.fdn = *reinterpret_cast<const uint32_t*>(d.flowdir + off + dn);
  r.wl = d.cw[off + lf];
  r.wr = d.cw[off + rt];
  r.fl = d.flowdir[off + lf];
  r.fr = d.flowdir[off + rt];
  return true;
}

__device__ __forceinline__ void flow_gather4(const Dev& d, const WorldParams& wp, uint32_t c0, uint32_t n,
                                             const int own[4], uint32_t fd, bool rows, const FlowRows& r,
                                             int out[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) out[j] = byte_of(fd, j) < 0 ? own[j] : 0;
  if (rows) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // the neighbour above (facing 0) leads here if it flows down (2), the one to
      // the right (1) if it flows left (3), below (2) if up (0), left (3) if right (1)
      if (byte_of(r.fu, j) == 2) out[j] += r.wu[j];
      if ((j < 3 ? byte_of(fd, j + 1) : r.fr) == 3) out[j] += j < 3 ? own[j + 1] : r.wr;
      if (byte_of(r.fdn, j) == 0) out[j] += r.wd[j];
      if ((j > 0 ? byte_of(fd, j - 1) : r.fl) == 1) out[j] += j > 0 ? own[j - 1] : r.wl;
    }
  } else {
    for (uint32_t j = 0; j < n; ++j) {
#pragma unroll
      for (int dd = 0; dd < 4; ++dd) {
        const uint32_t nb = wp.cell_off + neighbour(wp, c0 + j, dd, +1);
        if (d.flowdir[nb] == ((dd + 2) & 3)) out[j] += d.cw[nb];
      }
    }
  }
}

// The ecology's cell pass over tile tl, four consecutive cells per thread and pass
// (tile starts are multiples of 4): photosynthesis, one energy unit with
// probability min(1, rate * biomass) on cells holding biomass below the energy
// ceiling (the threshold in exact integers; the four cells' draws are the four
// outputs of one Philox block); the strikes of this step cleared (they have been
// counted); with terrain, the water's flow gathered into cw_next (the window-word
// pass copies it back once every cell has read the old layer).  Adds the
// photosynthesised units to grown and the grid totals of energy, water and biomass
// to total, wsum, bsum.
__device__ __forceinline__ void ecology_cells(const Dev& d, const WorldParams& wp, const eco_ecology& e, const Tile tl,
                                              uint32_t step, unsigned long long& grown, unsigned long long& total,
                                              unsigned long long& wsum, unsigned long long& bsum) {
  for (uint32_t i = 4 * threadIdx.x; i < tl.count; i += 4 * blockDim.x) {
    const uint32_t c0 = tl.start + i, n = min(4u, tl.count - i), g = wp.cell_off + c0;
    int b[4], en[4], wv[4];
    load_cells4(d.cb + g, b);
    load_cells4(d.ce + g, en);
    load_cells4(d.cw + g, wv);
    const uint32_t fd = d.rock ? *reinterpret_cast<const uint32_t*>(d.flowdir + g) : 0u;
    FlowRows fr{};   // the flow's neighbour rows, loaded with the cells' own values
    const bool rows = d.rock && flow_rows_load(d, wp, c0, n, fr);
    bool any = false;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) any |= j < n && b[j] > 0 && en[j] < e.cell_energy_max;
    if (any) {
      const uint4 x = regrow_draws(wp, c0 >> 2, step);
      bool grew = false;
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j)
        if (j < n && b[j] > 0 && en[j] < e.cell_energy_max &&
            (uint64_t)word_of(x, (int)j) < photo_threshold(e.photo_rate, b[j])) {
          ++en[j];
          ++grown;
          grew = true;
        }
      if (grew) store_cells4(d.ce + g, n, en);
    }
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
      if (j < n) {
        total += (unsigned long long)(uint32_t)en[j];
        wsum += (unsigned long long)(uint32_t)wv[j];
        bsum += (unsigned long long)(uint32_t)b[j];
      }
    if (wp.attack) {
      if (n == 4) {
        *reinterpret_cast<uint4*>(d.mark + g) = make_uint4(0u, 0u, 0u, 0u);
      } else {
        for (uint32_t j = 0; j < n; ++j) d.mark[g + j] = 0u;
      }
    }
    if (d.rock) {
      int nw[4];
      flow_gather4(d, wp, c0, n, wv, fd, rows, fr, nw);
      store_cells4(d.cw_next + g, n, nw);
    }
  }
}

__device__ __forceinline__ void regrow_tile(const Dev& d, const TileScratch& ts, uint32_t tile,
                                            unsigned long long* cnt) {
  const Tile tl = ts.cell_tiles[tile];
  const WorldParams wp = d.wp[tl.world];
  const uint32_t step = (uint32_t)d.wv[tl.world].step;
  if (d.ep) {   // ecology: photosynthesis, strikes, flow; the tile's grid totals for the statistics
    unsigned long long grown = 0, total = 0, wsum = 0, bsum = 0;
    ecology_cells(d, wp, d.ep[tl.world], tl, step, grown, total, wsum, bsum);
    wave_add_u64(grown, &cnt[0]);
    wave_add_u64(total, &cnt[1]);
    wave_add_u64(wsum, &cnt[2]);
    wave_add_u64(bsum, &cnt[3]);
    __syncthreads();
    if (threadIdx.x < kCellPart) ts.part_cell[tile * kCellPart + threadIdx.x] = cnt[threadIdx.x];
    return;
  }
  regrow_cells(d, wp, tl, step, cnt);
  __syncthreads();
  if (threadIdx.x < kCellPart) ts.part_cell[tile * kCellPart + threadIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_birth_claim_regrow(Dev d, TileScratch ts, uint32_t n_actions) {
  __shared__ uint32_t blocked;
  __shared__ unsigned long long cnt[kCellPart];
  if (threadIdx.x == 0) blocked = 0;
  if (threadIdx.x < kCellPart) cnt[threadIdx.x] = 0;
  __syncthreads();
  if (blockIdx.x < ts.n_slot_tiles) birth_claim_tile(d, ts, blockIdx.x, n_actions, &blocked);
  else regrow_tile(d, ts, blockIdx.x - ts.n_slot_tiles, cnt);
}

// Birth ranking, pass 1 (slot tiles): mark the claim winners; count claims,
// winners and free slots of the tile.
__global__ __launch_bounds__(kSlotTile) void k_birth_rank_count(Dev d, TileScratch ts) {
  __shared__ uint32_t cnt[3];
  if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
  __syncthreads();
  const Tile tl = ts.slot_tiles[blockIdx.x];
  const WorldParams wp = d.wp[tl.world];
  if (threadIdx.x < tl.count) {
    const uint32_t slot = wp.slot_off + tl.start + threadIdx.x;
    const uint8_t fl = d.flags[slot];
    if (fl & kBirthClaim) {
      count_lanes(&cnt[0]);
      if (d.claim[wp.cell_off + d.tgt[slot]] == slot) {
        d.flags[slot] = fl | kBirthWon;
        count_lanes(&cnt[1]);
      }
    }
    if (!(fl & kAlive)) count_lanes(&cnt[2]);
  }
  __syncthreads();
  if (threadIdx.x < 3) ts.scan[blockIdx.x * 4 + threadIdx.x] = cnt[threadIdx.x];
}

// Sum over the world's tiles [lo, hi) of pass-1 counter c (ts.scan[t][c]); all
// threads of the block get the sum.
template <int NT>
__device__ __forceinline__ uint32_t tiles_sum(const TileScratch& ts, uint32_t lo, uint32_t hi, int c,
                                              unsigned long long* red64, uint32_t* bcast) {
  uint32_t v = 0;
  for (uint32_t t = lo + threadIdx.x; t < hi; t += NT) v += ts.scan[t * 4 + c];
  const unsigned long long tot = block_sum_u64<NT>(v, red64);
  if (threadIdx.x == 0) *bcast = (uint32_t)tot;
  __syncthreads();
  const uint32_t r = *bcast;
  __syncthreads();
  return r;
}

// Birth ranking, pass 2 (slot tiles): winner k of the world (slot order) is
// recorded as bparent[k], free slot f (ascending) as freel[f].  A tile's
// offsets are the counts of the world's earlier tiles (pass 1), summed here;
// the world's last tile also records the world's birth totals.  Claims of
// this step are cleared.
__global__ __launch_bounds__(kSlotTile) void k_birth_rank_write(Dev d, TileScratch ts) {
  __shared__ uint32_t red[kSlotTile / 64 + 1];
  __shared__ unsigned long long red64[kSlotTile / 64];
  __shared__ uint32_t bcast;
  const Tile tl = ts.slot_tiles[blockIdx.x];
  const uint32_t w = tl.world;
  const WorldParams wp = d.wp[w];
  const uint32_t t0 = ts.tile_rng[4 * w], t1 = ts.tile_rng[4 * w + 1];
  const uint32_t ow = tiles_sum<kSlotTile>(ts, t0, blockIdx.x, 1, red64, &bcast);
  const uint32_t of = tiles_sum<kSlotTile>(ts, t0, blockIdx.x, 2, red64, &bcast);
  const bool in = threadIdx.x < tl.count;
  const uint32_t local = tl.start + threadIdx.x;
  const uint32_t slot = wp.slot_off + local;
  const uint8_t fl = in ? d.flags[slot] : (uint8_t)kAlive;
  uint32_t tot;
  const uint32_t rw = ow + block_exscan<kSlotTile>((fl & kBirthWon) ? 1u : 0u, red, &tot);
  const uint32_t rf = of + block_exscan<kSlotTile>((fl & kAlive) ? 0u : 1u, red, &tot);
  if (in) {
    if (fl & kBirthClaim) d.claim[wp.cell_off + d.tgt[slot]] = 0xFFFFFFFFu;
    if (fl & kBirthWon) d.bparent[wp.slot_off + rw] = (int)local;
    if (!(fl & kAlive)) d.freel[wp.slot_off + rf] = (int)local;
    if (fl & (kBirthClaim | kBirthWon)) d.flags[slot] = fl & kAlive;
  }
  if (blockIdx.x + 1 == t1) {  // the world's totals
    const uint32_t C = tiles_sum<kSlotTile>(ts, t0, t1, 0, red64, &bcast);
    const uint32_t Wn = tiles_sum<kSlotTile>(ts, t0, t1, 1, red64, &bcast);
    const uint32_t F = tiles_sum<kSlotTile>(ts, t0, t1, 2, red64, &bcast);
    if (threadIdx.x == 0) {
      const uint32_t nb = min(Wn, F);
      d.wv[w].n_births = nb;
      d.wv[w].n_win = Wn;
      d.cnt[w].births = nb;
      d.cnt[w].births_blocked_cell = C - Wn;
      d.cnt[w].births_blocked_capacity = Wn - nb;
    }
  }
}

// Prefix of per-world birth counts in LDS (same scheme as the live offsets).
__device__ __forceinline__ void birth_offsets(const WorldVar* __restrict__ wv, uint32_t n, uint32_t* off) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    const uint32_t per = (n + 63) / 64;
    const uint32_t lo = tid * per, hi = min(lo + per, n);
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; ++i) s += wv[i].n_births;
    const uint32_t inc = wave_scan(s);
    uint32_t run = inc - s;
    for (uint32_t i = lo; i < hi; ++i) {
      off[i] = run;
      run += wv[i].n_births;
    }
    if (tid == 63) off[n] = inc;
  }
  __syncthreads();
}

constexpr int kMaxWorlds = 1024;

// Unit u of an agent's master (16 bytes, four consecutive logical parameters):
// its Philox block (= first logical parameter / 4), layer (0..2 weights, 3..5
// biases), output row (first row for biases), k-block (the column quad in layer
// 2) and the number of its parameters that exist.  H = H1 = H2 is a power of
// two, so every index is a shift or a mask.
struct UnitPos {
  uint32_t blk, row, kb, nvalid;
  int layer;
};

template <int H>
__device__ __forceinline__ UnitPos unit_pos(const Layout& L, uint32_t u) {
  constexpr uint32_t LG = H == 32 ? 5 : (H == 64 ? 6 : 7);
  UnitPos r;
  r.nvalid = 4;
  r.kb = 0;
  if (u < L.u_b1) {                   // W1 [kb][row]: first parameter row D + 4 kb
    r.layer = 0; r.row = u & (H - 1); r.kb = u >> LG; r.blk = r.row * L.KB1 + r.kb;
  } else if (u < L.u_w2) {            // b1
    const uint32_t e = u - L.u_b1;
    r.layer = 3; r.row = 4 * e; r.blk = (L.p_b1 >> 2) + e;
  } else if (u < L.u_b2) {            // W2 [kb][row]: p_w2 + row H + 4 kb
    const uint32_t e = u - L.u_w2;
    r.layer = 1; r.row = e & (H - 1); r.kb = e >> LG; r.blk = (L.p_w2 >> 2) + r.row * (H / 4) + r.kb;
  } else if (u < L.u_w3) {            // b2
    const uint32_t e = u - L.u_b2;
    r.layer = 4; r.row = 4 * e; r.blk = (L.p_b2 >> 2) + e;
  } else if (u < L.u_b3) {            // W3 [row][H]: p_w3 + row H + 4 kb (rows >= A are padding)
    const uint32_t e = u - L.u_w3;
    r.layer = 2; r.row = e >> (LG - 2); r.kb = e & (H / 4 - 1); r.blk = (L.p_w3 >> 2) + e;
    r.nvalid = r.row < L.A ? 4u : 0u;
  } else {                            // b3, then the log temperature in slot A when it evolves
    const uint32_t e = u - L.u_b3, n3 = L.A + L.temp;
    r.layer = 5; r.row = 4 * e; r.blk = (L.p_b3 >> 2) + e;
    r.nvalid = r.row < n3 ? min(4u, n3 - r.row) : 0u;
  }
  return r;
}

// Streaming accesses of the weight blocks a birth reads once and writes once
// (non-temporal: no cache line is kept for them).
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 stream_load4(const float4* p) {
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
// The child's FP32 master; cached when it is read back for FP8 row scales (WDT 2).
template <int WDT>
__device__ __forceinline__ void stream_store4(float4* p, float a, float b, float c, float d) {
  if (WDT == 2) *p = make_float4(a, b, c, d);
  else __builtin_nontemporal_store(f32x4{a, b, c, d}, reinterpret_cast<f32x4*>(p));
}

// Storage copy of one unit's four master values (BF16 round-to-nearest-even;
// FP8: biases as FP32 here, weights after the row scales are known).
template <int WDT, int H>
__device__ __forceinline__ void store_unit(const Layout& L, uint8_t* sc, int layer, uint32_t row, uint32_t kb,
                                           const float (&v)[4], uint32_t* s_amax) {
  if (WDT == 1) {
    const uint32_t lo = bf16_rne(v[0]) | (bf16_rne(v[1]) << 16);
    const uint32_t hi = bf16_rne(v[2]) | (bf16_rne(v[3]) << 16);
    uint64_t off;
    if (layer == 0) off = L.s_w1 + ((uint64_t)(kb >> 1) * H + row) * 16 + (kb & 1) * 8;
    else if (layer == 1) off = L.s_w2 + ((uint64_t)(kb >> 1) * H + row) * 16 + (kb & 1) * 8;
    else if (layer == 2) off = L.s_w3 + ((uint64_t)row * H + 4 * kb) * 2;
    else off = L.s_b1 + (layer >= 4 ? L.s_b2 - L.s_b1 : 0u) + (layer >= 5 ? L.s_b3 - L.s_b2 : 0u) + (uint64_t)row * 2;
    *reinterpret_cast<uint2*>(sc + off) = make_uint2(lo, hi);   // half of a 16-byte block: cached
  } else if (WDT == 2) {
    if (layer < 3) {
      const uint32_t r = layer == 0 ? row : (layer == 1 ? H + row : 2 * H + row);
      const float mx = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
      atomicMax(&s_amax[r], __float_as_uint(mx));
    } else {
      const uint32_t base = L.s_b1 + (layer >= 4 ? L.s_b2 - L.s_b1 : 0u) + (layer >= 5 ? L.s_b3 - L.s_b2 : 0u);
      *reinterpret_cast<float4*>(sc + base + (uint64_t)row * 4) = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
}

// FP8 storage, after store_unit has gathered each row's amax in s_amax: the row
// scales, then the weights quantised with them (each thread re-reads the master
// units it wrote itself).
template <int H, int NT>
__device__ __forceinline__ void fp8_finish(const Layout& L, const float4* __restrict__ mc, uint8_t* sc,
                                           const uint32_t* s_amax, uint32_t tid) {
  const uint32_t nrows = 2 * H + L.R3;
  for (uint32_t r = tid; r < nrows; r += NT) {
    const float amax = __uint_as_float(s_amax[r]);
    const float scale = amax > 0.0f ? amax / 448.0f : 1.0f;
    uint64_t off;
    if (r < H) off = L.s_sc1 + (uint64_t)r * 4;
    else if (r < 2 * H) off = L.s_sc2 + (uint64_t)(r - H) * 4;
    else off = L.s_sc3 + (uint64_t)(r - 2 * H) * 4;
    *reinterpret_cast<float*>(sc + off) = scale;
  }
  // W1: the four k-blocks of one 16-byte storage block of a row (k-blocks 4j .. 4j + 3,
  // the missing ones of a row's last block zero) in one thread, written whole
  constexpr uint32_t LG = H == 32 ? 5 : (H == 64 ? 6 : 7);
  const uint32_t KB1 = L.KB1, nquads = ((KB1 + 3) >> 2) * H;
#pragma unroll 1
  for (uint32_t q = tid; q < nquads; q += NT) {
    const uint32_t row = q & (H - 1), j = q >> LG;
    const float amax = __uint_as_float(s_amax[row]);
    const float scale = amax > 0.0f ? amax / 448.0f : 1.0f;
    uint32_t wq[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const uint32_t kb = 4 * j + t;
      wq[t] = 0u;
      if (kb < KB1) {
        const float4 m4 = mc[kb * H + row];
        wq[t] = fp8_rne_sat(m4.x / scale) | (fp8_rne_sat(m4.y / scale) << 8) | (fp8_rne_sat(m4.z / scale) << 16) |
                (fp8_rne_sat(m4.w / scale) << 24);
      }
    }
    typedef unsigned int u32x4s __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(u32x4s{wq[0], wq[1], wq[2], wq[3]},
                                reinterpret_cast<u32x4s*>(sc + L.s_w1 + ((uint64_t)j * H + row) * 16));
  }
  for (uint32_t u = L.u_b1 + tid; u < L.u_b3; u += NT) {
    const UnitPos up = unit_pos<H>(L, u);
    const int layer = up.layer;
    const uint32_t row = up.row, kb = up.kb;
    if (layer >= 3) continue;
    const uint32_t r = layer == 0 ? row : (layer == 1 ? H + row : 2 * H + row);
    const float amax = __uint_as_float(s_amax[r]);
    const float scale = amax > 0.0f ? amax / 448.0f : 1.0f;
    const float4 m4 = mc[u];
    const uint32_t q = fp8_rne_sat(m4.x / scale) | (fp8_rne_sat(m4.y / scale) << 8) |
                       (fp8_rne_sat(m4.z / scale) << 16) | (fp8_rne_sat(m4.w / scale) << 24);
    uint64_t off;
    if (layer == 0) off = L.s_w1 + ((uint64_t)(kb >> 2) * H + row) * 16 + (kb & 3) * 4;
    else if (layer == 1) off = L.s_w2 + ((uint64_t)(kb >> 2) * H + row) * 16 + (kb & 3) * 4;
    else off = L.s_w3 + (uint64_t)row * H + 4 * kb;
    *reinterpret_cast<uint32_t*>(sc + off) = q;
  }
}

// Child master = parent master + sigma z (Sec. 3.3 mutation of every parameter),
// z standard normal from the parent's Philox stream (parent slot, step, MUTATE,
// block); the storage copy re-quantised from it; the child's |theta|^2.  One
// block of 256 threads per child.
template <int WDT, int H, int NT>
__device__ void mutate_child(const Dev& d, const Layout& L, const WorldParams& wp, uint32_t child, uint32_t parent,
                             uint32_t rng_slot, uint32_t step, const double2* tab, uint32_t* s_amax,
                             double* s_red) {
  const uint32_t tid = threadIdx.x;
  const float4* __restrict__ mp = reinterpret_cast<const float4*>(d.master + (uint64_t)parent * L.mstride);
  float4* __restrict__ mc = reinterpret_cast<float4*>(d.master + (uint64_t)child * L.mstride);
  uint8_t* sc = d.store + (uint64_t)child * L.sstride;
  if (WDT == 2) {
    for (uint32_t i = tid; i < 2 * H + L.R3; i += NT) s_amax[i] = 0u;
    __syncthreads();
  }
  const double sigma = (double)wp.sigma;
  const uint32_t key0 = wp.key0, key1 = wp.key1;
  if (L.colour && tid == 0) {
    // colour trait: the parent's plus sigma N(0,1) per channel
    double z[4];
    gauss4(wp, rng_slot, step, ST_COLOUR_MUTATE, 0u, tab, z);
    const float4 pc = d.colour[parent];
    d.colour[child] = make_float4((float)__builtin_fma(sigma, z[0], (double)pc.x),
                                  (float)__builtin_fma(sigma, z[1], (double)pc.y),
                                  (float)__builtin_fma(sigma, z[2], (double)pc.z), 0.0f);
  }
  double tsum = 0.0;
  auto unit = [&](uint32_t u, const UnitPos& up) {
    float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (up.nvalid > 0) {
      const float4 p4 = stream_load4(mp + u);
      const float pv[4] = {p4.x, p4.y, p4.z, p4.w};
      double z[4];
      gauss4k(key0, key1, rng_slot, step, ST_MUTATE, up.blk, tab, z);
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = (i < (int)up.nvalid) ? (float)__builtin_fma(sigma, z[i], (double)pv[i]) : 0.0f;
    }
    stream_store4<WDT>(mc + u, v[0], v[1], v[2], v[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) tsum += (double)v[i] * (double)v[i];
    store_unit<WDT, H>(L, sc, up.layer, up.row, up.kb, v, s_amax);
  };
  // W1 (most of the units) without the layer decode, then the other layers
  constexpr uint32_t LG = H == 32 ? 5 : (H == 64 ? 6 : 7);
  const uint32_t ub1 = L.u_b1;
  if (WDT == 1) {
    // BF16: the two units of one 16-byte storage block (k-blocks 2j and 2j + 1 of a
    // row) in one thread, so that the block is written whole and, like the
    // master, streamed past the caches (the second half of a row's last block is
    // padding when the row has an odd number of k-blocks: zero)
    const uint32_t KB1 = L.KB1, npairs = ((KB1 + 1) >> 1) * H;
#pragma unroll 1
    for (uint32_t q = tid; q < npairs; q += NT) {
      const uint32_t row = q & (H - 1), j = q >> LG, kb0 = 2 * j;
      const bool two = kb0 + 1 < KB1;
      const uint32_t u0 = kb0 * H + row, u1 = u0 + H;
      const float4 a = stream_load4(mp + u0);
      const float4 b = two ? stream_load4(mp + u1) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      const float pa[4] = {a.x, a.y, a.z, a.w}, pb[4] = {b.x, b.y, b.z, b.w};
      float va[4], vb[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      double z[4];
      gauss4k(key0, key1, rng_slot, step, ST_MUTATE, row * KB1 + kb0, tab, z);
#pragma unroll
      for (int i = 0; i < 4; ++i) va[i] = (float)__builtin_fma(sigma, z[i], (double)pa[i]);
      if (two) {
        gauss4k(key0, key1, rng_slot, step, ST_MUTATE, row * KB1 + kb0 + 1, tab, z);
#pragma unroll
        for (int i = 0; i < 4; ++i) vb[i] = (float)__builtin_fma(sigma, z[i], (double)pb[i]);
        stream_store4<WDT>(mc + u1, vb[0], vb[1], vb[2], vb[3]);
      }
      stream_store4<WDT>(mc + u0, va[0], va[1], va[2], va[3]);
#pragma unroll
      for (int i = 0; i < 4; ++i) tsum += (double)va[i] * (double)va[i] + (double)vb[i] * (double)vb[i];
      typedef unsigned int u32x4s __attribute__((ext_vector_type(4)));
      const u32x4s blk = {bf16_rne(va[0]) | (bf16_rne(va[1]) << 16), bf16_rne(va[2]) | (bf16_rne(va[3]) << 16),
                          bf16_rne(vb[0]) | (bf16_rne(vb[1]) << 16), bf16_rne(vb[2]) | (bf16_rne(vb[3]) << 16)};
      __builtin_nontemporal_store(blk, reinterpret_cast<u32x4s*>(sc + L.s_w1 + ((uint64_t)j * H + row) * 16));
    }
  }
  float4 next = (WDT != 1 && tid < ub1) ? stream_load4(mp + tid) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll 1
  for (uint32_t u = WDT == 1 ? ub1 : tid; u < ub1; u += NT) {
    const float4 p4 = next;   // this unit's parent values, loaded one unit ahead
    if (u + NT < ub1) next = stream_load4(mp + u + NT);
    const uint32_t row = u & (H - 1), kb = u >> LG;
    const float pv[4] = {p4.x, p4.y, p4.z, p4.w};
    double z[4];
    gauss4k(key0, key1, rng_slot, step, ST_MUTATE, row * L.KB1 + kb, tab, z);
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = (float)__builtin_fma(sigma, z[i], (double)pv[i]);
    stream_store4<WDT>(mc + u, v[0], v[1], v[2], v[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) tsum += (double)v[i] * (double)v[i];
    store_unit<WDT, H>(L, sc, 0, row, kb, v, s_amax);
  }
#pragma unroll 1
  for (uint32_t u = L.u_b1 + tid; u < L.u_end; u += NT) unit(u, unit_pos<H>(L, u));
  if (WDT == 2) {
    __syncthreads();
    fp8_finish<H, NT>(L, mc, sc, s_amax, tid);
  }
  const double t = block_sum_f64<NT>(tsum, s_red);
  if (tid == 0) d.trait[child] = t;
}

// Birth k of world w (the block's NT threads): the parent bparent[k] places
// its child in the free slot freel[k] (Sec. 3.2 reproduce, Sec. 3.3 mutation).
template <int WDT, int H, int NT>
__device__ __forceinline__ void commit_birth(const Dev& d, const Layout& L, uint32_t w, const WorldParams& wp,
                                             uint32_t k, uint32_t step, const double2* tab, uint32_t* s_amax,
                                             double* s_red) {
  const uint32_t p_local = (uint32_t)d.bparent[wp.slot_off + k];
  const uint32_t c_local = (uint32_t)d.freel[wp.slot_off + k];
  const uint32_t pg = wp.slot_off + p_local, cg = wp.slot_off + c_local;
  if (threadIdx.x == 0) {
    const int t = d.tgt[pg];
    d.energy[pg] -= wp.e_child;
    d.flags[cg] = kAlive;
    d.pos[cg] = t;
    d.occ[wp.cell_off + t] = (int)c_local;
    d.facing[cg] = d.facing[pg];
    d.energy[cg] = wp.e_child;
    d.age[cg] = 0;
    d.uid[cg] = d.wv[w].uid_next + k;
    d.puid[cg] = d.uid[pg];
    if (d.ep) {   // ecology: the parent gives water and biomass; the child starts at hp_child
      const eco_ecology& e = d.ep[w];
      d.water[pg] -= e.w_child;
      d.biomass[pg] -= e.b_child;
      d.water[cg] = e.w_child;
      d.biomass[cg] = e.b_child;
      d.hp[cg] = e.hp_child;
    }
  }
  mutate_child<WDT, H, NT>(d, L, wp, cg, pg, p_local, step, tab, s_amax, s_red);
  __syncthreads();
}

// One block per birth (persistent over all worlds' births).  Six waves per SIMD
// (five with a BF16 or FP8 copy to write) fit without spilling; the noise
// arithmetic of the other waves hides each wave's parent reads.
template <int WDT, int H>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WDT == 0 ? 6 : 5))) void k_birth_commit(Dev d, Layout L) {
  __shared__ uint32_t off[kMaxWorlds + 1];
  __shared__ uint32_t s_amax[128 + 128 + 16];
  __shared__ double s_red[4];
  __shared__ double2 tab[kTrigTable];
  birth_offsets(d.wv, d.n_worlds, off);
  const uint32_t total = off[d.n_worlds];
  if (blockIdx.x >= total) return;   // no birth for this block (the whole launch, in a step without births)
  load_trig(d.trig, tab);
  for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
    const uint32_t w = find_world(off, d.n_worlds, g);
    const WorldParams wp = d.wp[w];
    commit_birth<WDT, H, 256>(d, L, w, wp, g - off[w], (uint32_t)d.wv[w].step, tab, s_amax, s_red);
  }
}

// Trait moments of a group of agents: count, mean and the sum of squared
// deviations from that mean.  Two groups combine by the pairwise update of
// Chan, Golub and LeVeque (1979): with delta = mean_b - mean_a and n = n_a + n_b,
// mean = mean_a + delta n_b / n and M2 = M2_a + M2_b + delta^2 n_a n_b / n, which
// never subtracts two large sums (the variance of the whole is M2 / n).
struct Moments {
  double n, mean, m2;
};

__device__ __forceinline__ Moments merge_moments(const Moments& a, const Moments& b) {
  if (b.n == 0.0) return a;
  if (a.n == 0.0) return b;
  const double n = a.n + b.n, delta = b.mean - a.mean;
  return Moments{n, a.mean + delta * (b.n / n), a.m2 + b.m2 + delta * delta * (a.n * b.n / n)};
}

// Merge of one Moments per thread over the block, in a fixed order (a tree within
// each wave, then the waves in order); the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ Moments block_merge_moments(Moments m, double (*red)[3]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const Moments o{__shfl_down(m.n, d), __shfl_down(m.mean, d), __shfl_down(m.m2, d)};
    if (lane < d) m = merge_moments(m, o);
  }
  if (lane == 0) {
    red[wave][0] = m.n;
    red[wave][1] = m.mean;
    red[wave][2] = m.m2;
  }
  __syncthreads();
  Moments t{0.0, 0.0, 0.0};
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) t = merge_moments(t, Moments{red[i][0], red[i][1], red[i][2]});
  __syncthreads();
  return t;  // valid in thread 0
}

// Compaction, pass 1 (slot tiles): live count, energy sum and the trait moments of
// the tile (its mean, then the squared deviations from it: two passes over the
// tile's values, which stay in registers).
__global__ __launch_bounds__(kSlotTile) void k_compact_count(Dev d, TileScratch ts, int only_world) {
  __shared__ unsigned long long red64[kSlotTile / 64];
  __shared__ double redf[kSlotTile / 64];
  __shared__ double bcastf;
  const Tile tl = ts.slot_tiles[blockIdx.x];
  if (only_world >= 0 && (int)tl.world != only_world) return;
  const WorldParams wp = d.wp[tl.world];
  bool alive = false;
  long long e = 0;
  double t = 0.0;
  if (threadIdx.x < tl.count) {
    const uint32_t slot = wp.slot_off + tl.start + threadIdx.x;
    alive = d.flags[slot] & kAlive;
    if (alive) {
      e = d.energy[slot];
      t = d.trait[slot];
    }
  }
  const unsigned long long n = block_sum_u64<kSlotTile>(alive ? 1ull : 0ull, red64);
  const unsigned long long es = block_sum_u64<kSlotTile>((unsigned long long)e, red64);
  const double s1 = block_sum_f64<kSlotTile>(t, redf);
  if (threadIdx.x == 0) bcastf = n ? s1 / (double)n : 0.0;
  __syncthreads();
  const double tile_mean = bcastf;
  const double dv = alive ? t - tile_mean : 0.0;
  const double m2 = block_sum_f64<kSlotTile>(dv * dv, redf);
  if (d.ep) {   // ecology: water, biomass and health carried by the tile's live agents
    const uint32_t slot = wp.slot_off + tl.start + threadIdx.x;
    const bool on = alive && threadIdx.x < tl.count;
    const unsigned long long ws = block_sum_u64<kSlotTile>(on ? (unsigned long long)d.water[slot] : 0ull, red64);
    const unsigned long long bs = block_sum_u64<kSlotTile>(on ? (unsigned long long)d.biomass[slot] : 0ull, red64);
    const unsigned long long hs = block_sum_u64<kSlotTile>(on ? (unsigned long long)d.hp[slot] : 0ull, red64);
    if (threadIdx.x == 0) {
      ts.ecosum[3 * blockIdx.x] = ws;
      ts.ecosum[3 * blockIdx.x + 1] = bs;
      ts.ecosum[3 * blockIdx.x + 2] = hs;
    }
  }
  if (threadIdx.x == 0) {
    ts.scan[blockIdx.x * 4 + 3] = (uint32_t)n;
    ts.esum[blockIdx.x] = (long long)es;
    ts.tmean[blockIdx.x] = tile_mean;
    ts.tm2[blockIdx.x] = m2;
  }
}

// Window channels of every cell at the start of a step (Sec. 3.2 sensors, App. F
// layout), one byte per cell: bit 0 agent present, bit 1 resource present, bit 2
// wall (worlds with walls only), bits 3..5 the occupant's energy bin
// min(floor(8 E / e_repro), 7), built at the end of each step (and of init and
// state writes) for the next one.  The policy kernel's window gather then reads one
// byte per cell instead of the occupancy, resource and wall arrays plus a
// dependent read of each occupant's energy.  Threads take 4 consecutive cells
// (cell_off and tile starts are multiples of 4); a ragged tail goes cell by cell.
// The cell's resource and wall bits of its sense byte.
__device__ __forceinline__ uint32_t cell_sense(const WorldParams& wp, uint32_t r, uint32_t wl) {
  return (r != 0 ? 2u : 0u) | (wp.has_walls && wl != 0 ? 4u : 0u);
}

// An occupant's bits of the sense byte: the agent bit and its energy bin
// (the number of b in 1..7 with 8 E >= b e_repro).
__device__ __forceinline__ uint32_t agent_sense(const WorldParams& wp, int energy) {
  const long long e8 = (long long)energy * 8;
  uint32_t eb = 0;
#pragma unroll
  for (int b = 1; b < 8; ++b) eb += (e8 >= (long long)b * wp.e_repro) ? 1u : 0u;
  return 1u | (eb << 3);
}

__device__ __forceinline__ uint32_t sense_of(const WorldParams& wp, const Dev& d, int o, uint32_t r, uint32_t wl) {
  const uint32_t v = cell_sense(wp, r, wl);
  return o >= 0 ? v | agent_sense(wp, d.energy[wp.slot_off + (uint32_t)o]) : v;
}

// Colour vision: the cell as others see it (occupant's colour, else a resource
// unit in green, else a wall in grey, else black; 8 bits per channel), with the
// cell's agent / resource / wall bits in the top byte for the move claim.
// round(clamp(c, 0, 1) * 255) with ties up, in exact integer arithmetic: a c in
// (0, 1) is M 2^-s with an integer M < 2^24 and s >= 24, so the result is
// floor((255 M + 2^(s-1)) / 2^s).
__device__ __forceinline__ uint32_t colour_byte(float c) {
  if (!(c > 0.0f)) return 0u;   // also NaN
  if (c >= 1.0f) return 255u;
  const uint32_t u = __float_as_uint(c);
  const uint32_t ex = u >> 23;   // c > 0: sign bit clear
  const uint64_t M = ex ? ((u & 0x7FFFFFu) | 0x800000u) : (u & 0x7FFFFFu);
  const int s = ex ? 150 - (int)ex : 149;   // c = M 2^-s, s >= 24
  if (s >= 64) return 0u;
  return (uint32_t)((255ull * M + (1ull << (s - 1))) >> s);
}

// col: the live agents' colour words by local slot, if the caller has them in LDS
// (else read from the colour trait).
__device__ __forceinline__ uint32_t colour_word(const float4 c) {
  return colour_byte(c.x) | (colour_byte(c.y) << 8) | (colour_byte(c.z) << 16);
}

__device__ __forceinline__ void cell_render_tile(const Dev& d, const Tile tl, const uint32_t* col = nullptr) {
  const WorldParams wp = d.wp[tl.world];
  for (uint32_t i = threadIdx.x; i < tl.count; i += blockDim.x) {
    const uint32_t cell = wp.cell_off + tl.start + i;
    const int o = d.occ[cell];
    const bool r = d.res[cell] != 0, wl = wp.has_walls && d.wall[cell] != 0;
    uint32_t q = 0u;
    if (o >= 0) {
      q = col ? col[o] : colour_word(d.colour[wp.slot_off + (uint32_t)o]);
    } else if (r) {
      q = 255u << 8;
    } else if (wl) {
      q = 0x808080u;
    }
    d.rgb[cell] = q | (((o >= 0 ? 1u : 0u) | (r ? 2u : 0u) | (wl ? 4u : 0u)) << 24);
  }
}

// Ecology: the cell's water, energy and biomass levels (capped at 255), or with
// colour vision the cell as others see it (occupant's colour, wall grey, else
// energy / biomass / water as red / green / blue); the agent / wall bits and the
// rock height in the top byte.  flowed != 0 (the end of a step with terrain):
// first take the water the step's flow left on the cell.  Four consecutive cells
// per thread and pass, their loads issued together.
__device__ __forceinline__ uint32_t sat255(int v) { return (uint32_t)min(max(v, 0), 255); }

__device__ __forceinline__ void cell_ecology_tile(const Dev& d, const WorldParams& wp, const Tile tl, int flowed,
                                                  const uint32_t* col = nullptr) {
  for (uint32_t i = 4 * threadIdx.x; i < tl.count; i += 4 * blockDim.x) {
    const uint32_t n = min(4u, tl.count - i), g = wp.cell_off + tl.start + i;
    int wv[4], o[4], ce[4], cb[4], rk[4] = {0, 0, 0, 0};
    const bool copy_back = flowed && d.rock;
    load_cells4((copy_back ? d.cw_next : d.cw) + g, wv);
    load_cells4(d.occ + g, o);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
      if (j >= n) o[j] = -1;   // past a ragged tail: no occupant read
    load_cells4(d.ce + g, ce);
    load_cells4(d.cb + g, cb);
    if (d.rock) load_cells4(d.rock + g, rk);
    const uint32_t wl4 = wp.has_walls ? *reinterpret_cast<const uint32_t*>(d.wall + g) : 0u;
    if (copy_back) store_cells4(d.cw + g, n, wv);   // after every load of the group is issued
    uint32_t q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool wl = ((wl4 >> (8 * j)) & 0xFFu) != 0;
      if (!d.colour) {
        q[j] = sat255(wv[j]) | (sat255(ce[j]) << 8) | (sat255(cb[j]) << 16);
      } else if (o[j] >= 0) {
        q[j] = col ? col[o[j]] : colour_word(d.colour[wp.slot_off + (uint32_t)o[j]]);
      } else if (wl) {
        q[j] = 0x808080u;
      } else {
        q[j] = sat255(16 * min(ce[j], 1 << 20)) | (sat255(64 * min(cb[j], 1 << 20)) << 8) |
               (sat255(16 * min(wv[j], 1 << 20)) << 16);
      }
      q[j] |= ((o[j] >= 0 ? 1u : 0u) | (wl ? 4u : 0u) | ((uint32_t)rk[j] << 3)) << 24;
    }
    store_cells4(reinterpret_cast<int32_t*>(d.rgb + g), n, reinterpret_cast<const int*>(q));
  }
}

__device__ __forceinline__ void cell_sense_tile(const Dev& d, const Tile tl) {
  const WorldParams wp = d.wp[tl.world];
  for (uint32_t i = 4 * threadIdx.x; i < tl.count; i += 4 * blockDim.x) {
    const uint32_t cell = wp.cell_off + tl.start + i;
    if (i + 4 <= tl.count) {
      const int4 o = *reinterpret_cast<const int4*>(d.occ + cell);
      const uint32_t r = *reinterpret_cast<const uint32_t*>(d.res + cell);
      const uint32_t wl = *reinterpret_cast<const uint32_t*>(d.wall + cell);
      const uint32_t v = sense_of(wp, d, o.x, r & 0xFFu, wl & 0xFFu) | sense_of(wp, d, o.y, (r >> 8) & 0xFFu, (wl >> 8) & 0xFFu) << 8 |
                         sense_of(wp, d, o.z, (r >> 16) & 0xFFu, (wl >> 16) & 0xFFu) << 16 |
                         sense_of(wp, d, o.w, r >> 24, wl >> 24) << 24;
      *reinterpret_cast<uint32_t*>(d.sense + cell) = v;
    } else {
      for (uint32_t c = cell; c < wp.cell_off + tl.start + tl.count; ++c)
        d.sense[c] = (uint8_t)sense_of(wp, d, d.occ[c], d.res[c], d.wall[c]);
    }
  }
}

// The step's statistics record of world w once its compaction counts are in
// (pass 1), and the clock advance unless init != 0 (init / state writes).  Run
// by the block of the world's last slot tile (NT threads).
template <int NT>
__device__ void world_finalize(const Dev& d, const TileScratch& ts, uint32_t w, int init) {
  __shared__ uint32_t red[NT / 64 + 1];
  __shared__ unsigned long long red64[NT / 64];
  __shared__ double redm[NT / 64][3];
  __shared__ unsigned long long s_cnt[kSlotPart + kCellPart];
  const uint32_t t0 = ts.tile_rng[4 * w], t1 = ts.tile_rng[4 * w + 1];
  const uint32_t nt = t1 - t0;
  const uint32_t per = (nt + NT - 1) / NT;
  const uint32_t lo = t0 + threadIdx.x * per, hi = min(lo + per, t1);
  uint32_t n = 0;
  long long es = 0;
  Moments tm{0.0, 0.0, 0.0};   // the trait moments of this thread's tiles, merged in tile order
  for (uint32_t t = lo; t < hi; ++t) {
    const uint32_t nl = ts.scan[t * 4 + 3];
    n += nl;
    es += ts.esum[t];
    tm = merge_moments(tm, Moments{(double)nl, ts.tmean[t], ts.tm2[t]});
  }
  uint32_t N;
  block_exscan<NT>(n, red, &N);
  const unsigned long long E = block_sum_u64<NT>((unsigned long long)es, red64);
  const Moments TM = block_merge_moments<NT>(tm, redm);
  unsigned long long eco_w = 0, eco_b = 0, eco_h = 0;   // ecology: carried water, biomass, health
  if (d.ep) {
    unsigned long long a = 0, b = 0, c = 0;
    for (uint32_t t = lo; t < hi; ++t) {
      a += ts.ecosum[3 * t];
      b += ts.ecosum[3 * t + 1];
      c += ts.ecosum[3 * t + 2];
    }
    eco_w = block_sum_u64<NT>(a, red64);
    eco_b = block_sum_u64<NT>(b, red64);
    eco_h = block_sum_u64<NT>(c, red64);
  }
  if (threadIdx.x < kSlotPart + kCellPart) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  if (!init) {
    // per-thread sums over its tiles, then wave sums, then one LDS add per wave
    // (slot counters count agents, below 2^31 per world; the grid totals are u64)
    uint32_t c[kSlotPart];
    unsigned long long cc[kCellPart];
#pragma unroll
    for (int k = 0; k < kSlotPart; ++k) c[k] = 0;
#pragma unroll
    for (int k = 0; k < kCellPart; ++k) cc[k] = 0;
    for (uint32_t t = lo; t < hi; ++t)
#pragma unroll
      for (int k = 0; k < kSlotPart; ++k) c[k] += ts.part_slot[t * kSlotPart + k];
    const uint32_t ct0 = ts.tile_rng[4 * w + 2], ct1 = ts.tile_rng[4 * w + 3];
    for (uint32_t t = ct0 + threadIdx.x; t < ct1; t += NT)
#pragma unroll
      for (int k = 0; k < kCellPart; ++k) cc[k] += ts.part_cell[t * kCellPart + k];
#pragma unroll
    for (int k = 0; k < kSlotPart; ++k) c[k] = wave_scan(c[k]);
#pragma unroll
    for (int k = 0; k < kCellPart; ++k) cc[k] = wave_scan(cc[k]);
    if ((threadIdx.x & 63) == 63) {
#pragma unroll
      for (int k = 0; k < kSlotPart; ++k) atomicAdd(&s_cnt[k], (unsigned long long)c[k]);
#pragma unroll
      for (int k = 0; k < kCellPart; ++k) atomicAdd(&s_cnt[kSlotPart + k], cc[k]);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    WorldVar& v = d.wv[w];
    eco_stats st = {};
    if (!init) {
      v.step += 1;
      v.uid_next += v.n_births;
      st.births = d.cnt[w].births;
      st.births_blocked_cell = d.cnt[w].births_blocked_cell + s_cnt[PC_BB_CELL];
      st.births_blocked_capacity = d.cnt[w].births_blocked_capacity;
      st.deaths = s_cnt[PC_DEATHS];
      st.killed = s_cnt[PC_KILLED];
      st.eaten = s_cnt[PC_EATEN];
      st.moves_ok = s_cnt[PC_MOVES_OK];
      st.moves_blocked = s_cnt[PC_MOVES_BLOCKED];
      for (int a = 0; a < 9; ++a) st.action_hist[a] = s_cnt[PC_HIST + a];
      st.regrown = s_cnt[kSlotPart + 0];
      st.resource_total = s_cnt[kSlotPart + 1];
      if (d.ep) {
        st.water_total = eco_w + s_cnt[kSlotPart + 2];
        st.biomass_total = eco_b + s_cnt[kSlotPart + 3];
      }
    }
    if (d.ep) st.hp_total = eco_h;   // (init records get the grid parts from k_resource_total)
    v.n_live = N;
    st.step = v.step;
    st.population = N;
    st.energy_total = (double)(long long)E;
    st.trait_mean = N ? TM.mean : 0.0;
    st.trait_var = N ? TM.m2 / (double)N : 0.0;
    d.ring[(uint64_t)w * kStatsRing + (v.step % kStatsRing)] = st;
  }
}

// Compaction, pass 2.  Slot-tile blocks: the tile's live slots at their
// offsets in the world's live list (offset = live counts of the world's earlier
// tiles, summed here); the world's last tile also writes the step's statistics.
// Blocks past the slot tiles build the sense bytes of one cell tile each for the
// next step (the grid is final here).  only_world >= 0 restricts both parts.
__global__ __launch_bounds__(kSlotTile) void k_compact_write(Dev d, TileScratch ts, int init, int only_world) {
  __shared__ uint32_t red[kSlotTile / 64 + 1];
  __shared__ unsigned long long red64[kSlotTile / 64];
  __shared__ uint32_t bcast;
  if (blockIdx.x >= ts.n_slot_tiles) {
    const Tile ct = ts.cell_tiles[blockIdx.x - ts.n_slot_tiles];
    if (only_world < 0 || (int)ct.world == only_world) {
      if (d.ep) cell_ecology_tile(d, d.wp[ct.world], ct, !init);
      else if (d.rgb) cell_render_tile(d, ct);
      else cell_sense_tile(d, ct);
    }
    return;
  }
  const Tile tl = ts.slot_tiles[blockIdx.x];
  if (only_world >= 0 && (int)tl.world != only_world) return;
  const uint32_t w = tl.world;
  const WorldParams wp = d.wp[w];
  const uint32_t t0 = ts.tile_rng[4 * w], t1 = ts.tile_rng[4 * w + 1];
  const uint32_t ol = tiles_sum<kSlotTile>(ts, t0, blockIdx.x, 3, red64, &bcast);
  const bool in = threadIdx.x < tl.count;
  const uint32_t local = tl.start + threadIdx.x;
  const bool alive = in && (d.flags[wp.slot_off + local] & kAlive);
  uint32_t tot;
  const uint32_t r = ol + block_exscan<kSlotTile>(alive ? 1u : 0u, red, &tot);
  if (alive) d.live[wp.slot_off + r] = (int)local;
  if (blockIdx.x + 1 == t1) world_finalize<kSlotTile>(d, ts, w, init);
}

// ---------------------------------------------------------------------------
// The step after the policy kernel for an object of one small world, in one
// block: moves, eating, costs and deaths, birth claims and regrowth (the
// ecology: photosynthesis, and with terrain the water's flow), the birth
// ranking, the births, the next live list with the statistics record, and the
// next step's window channels (the same per-agent and per-cell rules as the
// kernels above, with the world's scans done inside the block).  A small world's
// step is bound by the latency of its launches, and this replaces seven
// dependent launches by one.  A thread scans a contiguous range of slots, so
// every scan is one block-wide exclusive sum.  ECO: the world has the ecology
// (d.ep set); the single-resource instantiation carries none of the ecology's
// phases (behind a run-time test they made its step measurably slower).
// ---------------------------------------------------------------------------
template <int WDT, int H, bool ECO>
__global__ __launch_bounds__(1024) void k_step_small(Dev d, Layout L, uint32_t n_actions) {
  // threads; slots or cells per thread in one pass (one 4-byte load of bytes); passes over
  // the slots (the capacity is at most NT CH NP)
  constexpr int NT = 1024, CH = 4, NP = 2;
  static_assert(NT * CH * NP == ECO_SMALL_STEP_MAX_SLOTS, "the slot passes cover the largest object taken");
  __shared__ uint32_t cnt[kSlotPart];              // step counters (PC_*)
  __shared__ unsigned long long ccnt[kCellPart];   // regrown units, resource total (the ecology: grid energy), grid water, biomass
  __shared__ uint32_t blocked, any_claim;
  __shared__ unsigned long long rank_red[NT / 64];   // the ranking scan's wave totals
  __shared__ uint32_t live_red[NT / 64];             // the live list's wave counts
  __shared__ unsigned long long red64[NT / 64];      // the waves' energy sums
  __shared__ double m2_red[NT / 64];                 // the waves' sums of squared deviations
  __shared__ unsigned long long eco_red[3][NT / 64];  // the ecology: the waves' carried water, biomass, health
  __shared__ uint32_t s_amax[128 + 128 + 16];
  __shared__ double s_red[NT / 64];                  // the births' reductions, then the waves' trait sums
  __shared__ double2 tab[kTrigTable];
  // per cell: the agent bit and energy bin of its occupant after the step (0: none),
  // written from the live slots, read by the window-channel pass
  __shared__ __align__(16) uint8_t s_agent[ECO_SMALL_STEP_MAX_CELLS];
  // colour vision: the live agents' colour words by slot, written from the live
  // slots, read by the window-word pass (no occupant-then-colour lookup chain)
  __shared__ uint32_t s_col[ECO_SMALL_STEP_MAX_SLOTS];
  const uint32_t tid = threadIdx.x;
  // live-list entry tid, loaded together with the world's live count: the
  // thread's only agent when there are at most NT (the object's one world
  // starts at slot 0; the list's allocation holds total_slots entries)
  const int32_t live_tid = d.live[min(tid, d.total_slots - 1u)];
  if (tid < kSlotPart) cnt[tid] = 0;
  if (tid < kCellPart) ccnt[tid] = 0;
  if (tid == 0) blocked = any_claim = 0;
  __syncthreads();
  constexpr uint32_t w = 0;
  const WorldParams wp = d.wp[w];
  const uint32_t step = (uint32_t)d.wv[w].step, n_live = d.wv[w].n_live, cap = wp.cap, cells = wp.cells;
  const int32_t* live = d.live + wp.slot_off;
  // each thread's contiguous range of the live list
  const uint32_t per_l = (n_live + NT - 1) / NT;
  const uint32_t l0 = min(tid * per_l, n_live), l1 = min(l0 + per_l, n_live);
  // the flag bytes of slots b0 .. b0 + 3 (slot and cell ranges start at multiples of
  // 64 and their allocations end at one, so these 4-byte loads stay inside)
  auto flags4 = [&](uint32_t b0) { return *reinterpret_cast<const uint32_t*>(d.flags + wp.slot_off + b0); };
  const bool sense_bytes = d.rgb == nullptr;   // window channels as sense bytes (else rendered words)
  if (sense_bytes)
    for (uint32_t c0 = tid * 16; c0 < cells; c0 += NT * 16) *reinterpret_cast<uint4*>(s_agent + c0) = make_uint4(0, 0, 0, 0);

  // 1. moves, eating, costs and deaths of the step's live agents
  for (uint32_t i = l0; i < l1; ++i) {
    const uint32_t local = (uint32_t)(i == tid ? live_tid : live[i]);
    move_agent(d, wp, w, wp.slot_off + local, local, step + 1u, cnt);
  }
  __syncthreads();
  // 2. birth claims of the agents still alive; regrowth of every cell (4 per thread and pass)
  bool claimed = false;
  for (uint32_t i = l0; i < l1; ++i) claimed |= birth_claim_slot(d, wp, w, wp.slot_off + (uint32_t)live[i], n_actions, &blocked);
  if (claimed) any_claim = 1u;   // the same value from every claimant
  if constexpr (ECO) {   // the ecology: photosynthesis, strikes cleared, the flow gather; the grid totals
    unsigned long long grown = 0, total = 0, wsum = 0, bsum = 0;
    ecology_cells(d, wp, d.ep[w], Tile{w, 0u, cells, 0u}, step, grown, total, wsum, bsum);
    wave_add_u64(grown, &ccnt[0]);
    wave_add_u64(total, &ccnt[1]);
    wave_add_u64(wsum, &ccnt[2]);
    wave_add_u64(bsum, &ccnt[3]);
  } else {
    unsigned long long grown = 0, total = 0;
    for (uint32_t c0 = tid * CH; c0 < cells; c0 += NT * CH) {
      uint32_t* rp = reinterpret_cast<uint32_t*>(d.res + wp.cell_off + c0);
      const uint32_t v = *rp;
      const uint32_t nv = regrow_word(wp, c0, min((uint32_t)CH, cells - c0), v, step, grown, total);
      if (nv != v) *rp = nv;
    }
    wave_add_u64(grown, &ccnt[0]);
    wave_add_u64(total, &ccnt[1]);
  }
  __syncthreads();
  // 3. birth ranking, when any parent claimed a cell: the claim winners in slot
  // order (the live list's order) and the free slots in ascending order (the
  // recycled-slot free list; only its first Wn entries are used), both ranked by
  // one block scan of 16-bit counts packed in a u64 (winners, free slots of each
  // pass, claims; no field carries into the next: every total is at most 8,192).
  // The claimed cells are released right after the ranking, the claim flags by the
  // last pass over the slots.
  uint32_t Wn = 0, claims = 0, nb = 0;
  if (any_claim) {   // the same in every thread (written before the barrier above)
    uint32_t nw = 0, nc = 0;
    for (uint32_t i = l0; i < l1; ++i) {
      const uint32_t slot = wp.slot_off + (uint32_t)live[i];
      if (d.flags[slot] & kBirthClaim) {
        ++nc;
        if (d.claim[wp.cell_off + d.tgt[slot]] == slot) ++nw;
      }
    }
    uint32_t fm[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const uint32_t b0 = (p * NT + tid) * CH;
      fm[p] = 0;
      if (b0 < cap) {
        const uint32_t v = flags4(b0);
#pragma unroll
        for (int j = 0; j < CH; ++j)
          if (b0 + j < cap && !((v >> (8 * j)) & kAlive)) fm[p] |= 1u << j;
      }
    }
    static_assert(NP == 2, "the packed ranking scan holds two passes of free slots");
    unsigned long long rtot;
    const unsigned long long rex =
        block_exscan_u64<NT>((unsigned long long)nw | (unsigned long long)__builtin_popcount(fm[0]) << 16 |
                                 (unsigned long long)__builtin_popcount(fm[1]) << 32 | (unsigned long long)nc << 48,
                             rank_red, &rtot);
    Wn = (uint32_t)(rtot & 0xFFFFu);
    claims = (uint32_t)(rtot >> 48);
    uint32_t k = (uint32_t)(rex & 0xFFFFu);
    for (uint32_t i = l0; i < l1 && nw; ++i) {
      const uint32_t local = (uint32_t)live[i], slot = wp.slot_off + local;
      if ((d.flags[slot] & kBirthClaim) && d.claim[wp.cell_off + d.tgt[slot]] == slot) d.bparent[wp.slot_off + k++] = (int)local;
    }
    uint32_t F = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const uint32_t b0 = (p * NT + tid) * CH;
      uint32_t f = F + (uint32_t)((rex >> (16 * (p + 1))) & 0xFFFFu);
      for (uint32_t m = fm[p]; m && f < Wn; m &= m - 1) d.freel[wp.slot_off + f++] = (int)(b0 + __builtin_ctz(m));
      F += (uint32_t)((rtot >> (16 * (p + 1))) & 0xFFFFu);
    }
    nb = min(Wn, F);
    __syncthreads();
    // the claimed cells released (every claimant has read its cell's claim word;
    // the movers' winners released theirs in the move phase)
    for (uint32_t i = l0; i < l1; ++i) {
      const uint32_t slot = wp.slot_off + (uint32_t)live[i];
      if (d.flags[slot] & kBirthClaim) d.claim[wp.cell_off + d.tgt[slot]] = 0xFFFFFFFFu;
    }
  }
  // 4. the births, one at a time (the angle table of the mutation noise only when there are any)
  if (nb) load_trig(d.trig, tab);
  for (uint32_t b = 0; b < nb; ++b) commit_birth<WDT, H, NT>(d, L, w, wp, b, step, tab, s_amax, s_red);
  // 5. the next step's live list and the statistics record: energy exact in
  // integers, the trait moments of each wave in two passes over the values held
  // in registers, merged across waves.  One barrier gives every wave its offsets
  // in the live list (both passes' counts packed in a u32) and thread 0 the
  // waves' energy sums and trait moments.
  long long es = 0;
  double t[NP][CH], s1 = 0.0;
  uint32_t am[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const uint32_t b0 = (p * NT + tid) * CH;
    am[p] = 0;
    if (b0 < cap) {
      const uint32_t v = flags4(b0);
#pragma unroll
      for (int j = 0; j < CH; ++j)
        if (b0 + j < cap && ((v >> (8 * j)) & kAlive)) am[p] |= 1u << j;
      // the step's birth-claim flags cleared (a flag byte is 0 or alive, after the step)
      constexpr uint32_t claim_bits = 0x01010101u * (kBirthClaim | kBirthWon);
      if (v & claim_bits) *reinterpret_cast<uint32_t*>(d.flags + wp.slot_off + b0) = v & ~claim_bits;
    }
    // the four slots' traits and energies in 16-byte loads, whether alive or not
    // (they lie inside the allocations, which end at a multiple of 64 slots)
    static_assert(CH == 4, "one 16-byte load of energies per pass");
    double2 tv[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    int4 ev = make_int4(0, 0, 0, 0), pv = make_int4(0, 0, 0, 0);
    if (b0 < cap) {
      tv[0] = *reinterpret_cast<const double2*>(d.trait + wp.slot_off + b0);
      tv[1] = *reinterpret_cast<const double2*>(d.trait + wp.slot_off + b0 + 2);
      ev = *reinterpret_cast<const int4*>(d.energy + wp.slot_off + b0);
      if (sense_bytes) pv = *reinterpret_cast<const int4*>(d.pos + wp.slot_off + b0);
    }
    float4 cv[4];
    if (d.colour && b0 < cap) {
#pragma unroll
      for (int j = 0; j < CH; ++j) cv[j] = d.colour[wp.slot_off + b0 + j];
    }
    const double tj[4] = {tv[0].x, tv[0].y, tv[1].x, tv[1].y};
    const int ej[4] = {ev.x, ev.y, ev.z, ev.w}, pj[4] = {pv.x, pv.y, pv.z, pv.w};
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const bool on = (am[p] >> j) & 1u;
      t[p][j] = on ? tj[j] : 0.0;
      es += on ? ej[j] : 0;
      if (sense_bytes && on) s_agent[pj[j]] = (uint8_t)agent_sense(wp, ej[j]);   // one agent per cell
      if (d.colour && on) s_col[b0 + j] = colour_word(cv[j]);
    }

#pragma unroll
    for (int j = 0; j < CH; ++j) s1 += t[p][j];
  }
  const int lane = (int)(tid & 63u), wave = (int)(tid >> 6);
  const uint32_t own = (uint32_t)__builtin_popcount(am[0]) | (uint32_t)__builtin_popcount(am[1]) << 16;
  const uint32_t inc = wave_scan(own);
  const unsigned long long ew = wave_scan((unsigned long long)es);
  // the wave's trait moments in two passes over its values: count, mean, and the
  // sum of squared deviations from that mean (merged across waves by thread 0)
  const uint32_t wc = lane_value(inc, 63);
  const double n_w = (double)((wc & 0xFFFFu) + (wc >> 16));
  const double mean_w = n_w > 0.0 ? lane_value(wave_scan(s1), 63) / n_w : 0.0;
  double m2 = 0.0;
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int j = 0; j < CH; ++j)
      if ((am[p] >> j) & 1u) m2 += (t[p][j] - mean_w) * (t[p][j] - mean_w);
  m2 = wave_scan(m2);
  // the ecology: water, biomass and health carried by the live agents (after the
  // trait values are no longer needed)
  unsigned long long eco_w[3] = {0, 0, 0};
  if constexpr (ECO) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const uint32_t b0 = (p * NT + tid) * CH;
      if (b0 < cap) {
        const int4 wv4 = *reinterpret_cast<const int4*>(d.water + wp.slot_off + b0);
        const int4 bv4 = *reinterpret_cast<const int4*>(d.biomass + wp.slot_off + b0);
        const int4 hv4 = *reinterpret_cast<const int4*>(d.hp + wp.slot_off + b0);
        const int wj[4] = {wv4.x, wv4.y, wv4.z, wv4.w}, bj[4] = {bv4.x, bv4.y, bv4.z, bv4.w},
                  hj[4] = {hv4.x, hv4.y, hv4.z, hv4.w};
#pragma unroll
        for (int j = 0; j < CH; ++j)
          if ((am[p] >> j) & 1u) {
            eco_w[0] += (unsigned long long)wj[j];
            eco_w[1] += (unsigned long long)bj[j];
            eco_w[2] += (unsigned long long)hj[j];
          }
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) eco_w[k] = wave_scan(eco_w[k]);
  }
  if (lane == 63) {
    live_red[wave] = inc;
    red64[wave] = ew;
    s_red[wave] = mean_w;
    m2_red[wave] = m2;
    if constexpr (ECO) {
#pragma unroll
      for (int k = 0; k < 3; ++k) eco_red[k][wave] = eco_w[k];
    }
  }
  __syncthreads();
  // each wave's offsets in the live list (the waves' counts added the same way in
  // every wave, lane i reading wave i's)
  uint32_t ntot;
  const uint32_t before = waves_before<NT / 64>(lane < NT / 64 ? live_red[lane] : 0u, &ntot);
  const uint32_t N0 = ntot & 0xFFFFu, N = N0 + (ntot >> 16);
  const uint32_t ex = before + inc - own;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const uint32_t b0 = (p * NT + tid) * CH;
    uint32_t r = (p == 0 ? 0u : N0) + ((ex >> (16 * p)) & 0xFFFFu);
    for (uint32_t a = am[p]; a; a &= a - 1) d.live[wp.slot_off + r++] = (int)(b0 + __builtin_ctz(a));
  }
  if (tid == 0) {
    // the energy total exactly, the trait moments by the pairwise (Chan-Golub-LeVeque)
    // merge of the waves' in wave order
    unsigned long long E = 0;
    Moments tm{0.0, 0.0, 0.0};
    for (int i = 0; i < NT / 64; ++i) {
      E += red64[i];
      const uint32_t c = live_red[i];
      tm = merge_moments(tm, Moments{(double)((c & 0xFFFFu) + (c >> 16)), s_red[i], m2_red[i]});
    }
    const double mean = N ? tm.mean : 0.0, M2 = tm.m2;
    WorldVar& v = d.wv[w];
    v.n_births = nb;
    v.n_win = Wn;
    v.step += 1;
    v.uid_next += nb;
    v.n_live = N;
    d.cnt[w].births = nb;
    d.cnt[w].births_blocked_cell = claims - Wn;
    d.cnt[w].births_blocked_capacity = Wn - nb;
    eco_stats st = {};
    st.step = v.step;
    st.population = N;
    st.births = nb;
    st.births_blocked_cell = claims - Wn + blocked;
    st.births_blocked_capacity = Wn - nb;
    st.deaths = cnt[PC_DEATHS];
    st.killed = cnt[PC_KILLED];
    st.eaten = cnt[PC_EATEN];
    st.moves_ok = cnt[PC_MOVES_OK];
    st.moves_blocked = cnt[PC_MOVES_BLOCKED];
    for (int a = 0; a < 9; ++a) st.action_hist[a] = cnt[PC_HIST + a];
    st.regrown = ccnt[0];
    st.resource_total = ccnt[1];
    st.energy_total = (double)(long long)E;
    st.trait_mean = mean;
    st.trait_var = N ? M2 / (double)N : 0.0;
    if constexpr (ECO) {   // grid (the cell pass) plus carried (the live slots)
      unsigned long long ecot[3] = {0, 0, 0};
#pragma unroll 1
      for (int i = 0; i < NT / 64; ++i)
        for (int k = 0; k < 3; ++k) ecot[k] += eco_red[k][i];
      st.water_total = ecot[0] + ccnt[2];
      st.biomass_total = ecot[1] + ccnt[3];
      st.hp_total = ecot[2];
    }
    d.ring[(uint64_t)w * kStatsRing + (v.step % kStatsRing)] = st;
  }
  // the window channels of every cell for the next step (the grid is final)
  if (sense_bytes) {
    // the sense bytes: resource and wall bits of each cell, with its occupant's
    // agent bit and energy bin from s_agent (complete since the barrier above)
    for (uint32_t c0 = tid * 4; c0 < cells; c0 += NT * 4) {
      const uint32_t g = wp.cell_off + c0;
      const uint32_t r = *reinterpret_cast<const uint32_t*>(d.res + g);
      const uint32_t wl = *reinterpret_cast<const uint32_t*>(d.wall + g);
      const uint32_t ag = *reinterpret_cast<const uint32_t*>(s_agent + c0);
      uint32_t v = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        v |= (((ag >> (8 * j)) & 0xFFu) | cell_sense(wp, (r >> (8 * j)) & 0xFFu, (wl >> (8 * j)) & 0xFFu)) << (8 * j);
      if (c0 + 4 <= cells) {
        *reinterpret_cast<uint32_t*>(d.sense + g) = v;
      } else {
        for (uint32_t j = 0; c0 + j < cells; ++j) d.sense[g + j] = (uint8_t)(v >> (8 * j));
      }
    }
  } else if (ECO) {
    cell_ecology_tile(d, wp, Tile{w, 0u, cells, 0u}, 1, s_col);   // with terrain, the flowed water copied back first
  } else {
    cell_render_tile(d, Tile{w, 0u, cells, 0u}, s_col);
  }
}

// Rendered window words of one world's cells (after a colour write).
__global__ __launch_bounds__(256) void k_render(Dev d, const Tile* __restrict__ tiles, int only_world) {
  const Tile ct = tiles[blockIdx.x];
  if ((int)ct.world != only_world) return;
  if (d.ep) cell_ecology_tile(d, d.wp[ct.world], ct, 0);
  else cell_render_tile(d, ct);
}

// Terrain: each cell's way down, the lowest 4-neighbour if strictly lower (the
// first of N, E, S, W among equals), else -1.
__global__ __launch_bounds__(256) void k_flowdir(Dev d, const Tile* __restrict__ tiles, int only_world) {
  const Tile tl = tiles[blockIdx.x];
  if (only_world >= 0 && (int)tl.world != only_world) return;
  const WorldParams wp = d.wp[tl.world];
  for (uint32_t i = threadIdx.x; i < tl.count; i += blockDim.x) {
    const uint32_t c = tl.start + i;
    int best = -1, bh = d.rock[wp.cell_off + c];
    for (int dd = 0; dd < 4; ++dd) {
      const int h = d.rock[wp.cell_off + neighbour(wp, c, dd, +1)];
      if (h < bh) { bh = h; best = dd; }
    }
    d.flowdir[wp.cell_off + c] = (int8_t)best;
  }
}

// Resource total of each world (init / after state writes): one block per world.
__global__ __launch_bounds__(kScanThreads) void k_resource_total(Dev d, int only_world) {
  __shared__ unsigned long long red64[kScanThreads / 64];
  const uint32_t w = blockIdx.x;
  if (only_world >= 0 && (int)w != only_world) return;
  const WorldParams wp = d.wp[w];
  unsigned long long s = 0;
  eco_stats* rec = &d.ring[(uint64_t)w * kStatsRing + (d.wv[w].step % kStatsRing)];
  if (d.ep) {   // ecology: energy on the grid; water and biomass on the grid and in live agents
    unsigned long long sw = 0, sb = 0;
    for (uint32_t c = threadIdx.x; c < wp.cells; c += blockDim.x) {
      const uint32_t g = wp.cell_off + c;
      s += (unsigned long long)d.ce[g];
      sw += (unsigned long long)d.cw[g];
      sb += (unsigned long long)d.cb[g];
    }
    for (uint32_t j = threadIdx.x; j < wp.cap; j += blockDim.x) {
      const uint32_t g = wp.slot_off + j;
      if (d.flags[g] & kAlive) {
        sw += (unsigned long long)d.water[g];
        sb += (unsigned long long)d.biomass[g];
      }
    }
    const unsigned long long t = block_sum_u64<kScanThreads>(s, red64);
    const unsigned long long tw = block_sum_u64<kScanThreads>(sw, red64);
    const unsigned long long tb = block_sum_u64<kScanThreads>(sb, red64);
    if (threadIdx.x == 0) {
      rec->resource_total = t;
      rec->water_total = tw;
      rec->biomass_total = tb;
    }
    return;
  }
  for (uint32_t c = threadIdx.x; c < wp.cells; c += blockDim.x) s += d.res[wp.cell_off + c];
  const unsigned long long t = block_sum_u64<kScanThreads>(s, red64);
  if (threadIdx.x == 0) rec->resource_total = t;
}

// ---------------------------------------------------------------------------
// Init kernels
// ---------------------------------------------------------------------------
// Terrain height of local cell (x, y): bilinear blend, in exact integers with
// floor division, of the four surrounding values (0..31) of a torus lattice of
// NX x NY seeded values, NX = max(1, W / terrain_scale).
__device__ __forceinline__ int terrain_height(const WorldParams& wp, const eco_ecology& e, uint32_t x, uint32_t y) {
  const uint64_t W = wp.W, H = wp.H, L = (uint64_t)e.terrain_scale;
  const uint64_t NX = W / L > 0 ? W / L : 1, NY = H / L > 0 ? H / L : 1;
  const uint64_t ax = (uint64_t)x * NX, ay = (uint64_t)y * NY;
  const uint64_t i = ax / W, j = ay / H, fx = ax % W, fy = ay % H;
  const uint64_t i1 = (i + 1) % NX, j1 = (j + 1) % NY;
  const uint64_t v00 = draw32(wp, (uint32_t)(i + j * NX), 0u, ST_TERRAIN) >> 27;
  const uint64_t v10 = draw32(wp, (uint32_t)(i1 + j * NX), 0u, ST_TERRAIN) >> 27;
  const uint64_t v01 = draw32(wp, (uint32_t)(i + j1 * NX), 0u, ST_TERRAIN) >> 27;
  const uint64_t v11 = draw32(wp, (uint32_t)(i1 + j1 * NX), 0u, ST_TERRAIN) >> 27;
  const uint64_t num = v00 * (W - fx) * (H - fy) + v10 * fx * (H - fy) + v01 * (W - fx) * fy + v11 * fx * fy;
  return (int)(num / (W * H));
}

// floor(p * 2^32) clamped to [0, 2^32]: a 32-bit draw x is a Bernoulli(p) success iff x < it.
__device__ __forceinline__ uint64_t density_threshold(float p) {
  double t = floor((double)p * 4294967296.0);
  t = t < 0.0 ? 0.0 : (t > 4294967296.0 ? 4294967296.0 : t);
  return (uint64_t)t;
}

// Cell keys (for placement), initial resources, empty occupancy and claims.
__global__ __launch_bounds__(256) void k_init_cells(Dev d, const Tile* __restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const WorldParams wp = d.wp[tl.world];
  for (uint32_t i = threadIdx.x; i < tl.count; i += blockDim.x) {
    const uint32_t c = tl.start + i, g = wp.cell_off + c;
    const uint32_t key = draw32(wp, c, 0u, ST_CELLKEY);
    d.cellkeys[g] = ((unsigned long long)key << 32) | c;
    d.res[g] = ((uint64_t)draw32(wp, c, 0u, ST_RESINIT) < wp.density_thr) ? 1 : 0;
    if (d.ep) {   // ecology: water, energy, biomass sites from outputs 1..3 of the same block
      const eco_ecology& e = d.ep[tl.world];
      const uint4 x = philox10(c, 0u, ST_RESINIT, 0u, wp.key0, wp.key1);
      d.res[g] = 0;
      d.cw[g] = ((uint64_t)x.y < density_threshold(e.water_density)) ? e.water_site : 0;
      d.ce[g] = ((uint64_t)x.z < density_threshold(e.energy_density)) ? e.energy_site : 0;
      d.cb[g] = ((uint64_t)x.w < density_threshold(e.biomass_density)) ? e.biomass_site : 0;
      if (d.rock) {   // terrain: the rock layer, and the sea instead of water sites
        const int r = terrain_height(wp, e, c % wp.W, c / wp.W);
        d.rock[g] = r;
        d.cw[g] = r < e.sea_level ? (e.sea_level - r) * e.water_per_depth : 0;
      }
    }
    d.occ[g] = -1;
    d.claim[g] = 0xFFFFFFFFu;
    if (wp.attack) d.mark[g] = 0;
    d.wall[g] = 0;
  }
}

// Placement (Sec. 3.2: the initial population on distinct cells; slot j takes
// the cell with the j-th smallest (Philox key, cell) pair).  The keys are 32-bit
// uniform draws, so a world's cells are bucketed by the top bits of the key into
// 2^k buckets of about four cells each (counts, a per-world exclusive scan, a
// scatter), and each cell's rank is its bucket's start plus the number of cells
// of its bucket with a smaller (key, cell) pair.  Only ranks below n_init are
// written.  Init only, never on the step path.
struct PlaceInfo {
  uint32_t boff;    // first bucket of the world in the bucket arrays
  uint32_t shift;   // bucket = key >> shift (2^(32 - shift) buckets)
};

__device__ __forceinline__ uint32_t place_bucket(const PlaceInfo& pi, unsigned long long k64) {
  return pi.boff + (pi.shift >= 32 ? 0u : (uint32_t)(k64 >> 32) >> pi.shift);
}

// Bucket counts (cnt zeroed by the caller).
__global__ __launch_bounds__(256) void k_place_count(Dev d, const Tile* __restrict__ tiles,
                                                     const PlaceInfo* __restrict__ pinfo, uint32_t* cnt) {
  const Tile tl = tiles[blockIdx.x];
  const WorldParams wp = d.wp[tl.world];
  const PlaceInfo pi = pinfo[tl.world];
  for (uint32_t i = threadIdx.x; i < tl.count; i += blockDim.x)
    atomicAdd(&cnt[place_bucket(pi, d.cellkeys[wp.cell_off + tl.start + i])], 1u);
}

// Per world (one block each): start[b] = exclusive prefix of the counts over the
// world's buckets (start of world w's buckets at boff + w, one extra entry per
// world holding its total), and the counts cleared for the scatter's cursors.
__global__ __launch_bounds__(kScanThreads) void k_place_scan(const PlaceInfo* __restrict__ pinfo, uint32_t* cnt,
                                                             uint32_t* start) {
  __shared__ uint32_t red[kScanThreads / 64 + 1];
  const uint32_t w = blockIdx.x;
  const PlaceInfo pi = pinfo[w];
  const uint32_t nb = pinfo[w + 1].boff - pi.boff;
  const uint32_t per = (nb + kScanThreads - 1) / kScanThreads;
  const uint32_t lo = pi.boff + threadIdx.x * per, hi = min(lo + per, pi.boff + nb);
  uint32_t own = 0;
  for (uint32_t b = lo; b < hi; ++b) own += cnt[b];
  uint32_t total;
  uint32_t run = block_exscan<kScanThreads>(own, red, &total);
  for (uint32_t b = lo; b < hi; ++b) {
    const uint32_t c = cnt[b];
    start[b + w] = run;
    run += c;
    cnt[b] = 0;
  }
  if (threadIdx.x == 0) start[pi.boff + nb + w] = total;
}

// Each cell into its bucket (unordered within the bucket) of sorted[].
__global__ __launch_bounds__(256) void k_place_scatter(Dev d, const Tile* __restrict__ tiles,
                                                       const PlaceInfo* __restrict__ pinfo, uint32_t* cnt,
                                                       const uint32_t* __restrict__ start) {
  const Tile tl = tiles[blockIdx.x];
  const WorldParams wp = d.wp[tl.world];
  const PlaceInfo pi = pinfo[tl.world];
  for (uint32_t i = threadIdx.x; i < tl.count; i += blockDim.x) {
    const unsigned long long k = d.cellkeys[wp.cell_off + tl.start + i];
    const uint32_t b = place_bucket(pi, k);
    d.sorted[wp.cell_off + start[b + tl.world] + atomicAdd(&cnt[b], 1u)] = k;
  }
}

// Rank of each bucketed cell; ranks below n_init go to cellkeys[cell_off + rank].
__global__ __launch_bounds__(256) void k_place_rank(Dev d, const Tile* __restrict__ tiles,
                                                    const PlaceInfo* __restrict__ pinfo,
                                                    const uint32_t* __restrict__ start) {
  const Tile tl = tiles[blockIdx.x];
  const WorldParams wp = d.wp[tl.world];
  const PlaceInfo pi = pinfo[tl.world];
  for (uint32_t i = threadIdx.x; i < tl.count; i += blockDim.x) {
    const unsigned long long k = d.sorted[wp.cell_off + tl.start + i];
    const uint32_t b = place_bucket(pi, k) + tl.world;
    const uint32_t s0 = start[b], s1 = start[b + 1];
    if (s0 >= wp.n_init) continue;   // the whole bucket ranks past the initial population
    uint32_t r = s0;
    for (uint32_t q = s0; q < s1; ++q) r += d.sorted[wp.cell_off + q] < k ? 1u : 0u;
    if (r < wp.n_init) d.cellkeys[wp.cell_off + r] = k;
  }
}

// Slot j < n_init takes the j-th smallest (key, cell); all other slots are free.
__global__ __launch_bounds__(kSlotTile) void k_init_agents(Dev d, const Tile* __restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const WorldParams wp = d.wp[tl.world];
  if (threadIdx.x >= tl.count) return;
  const uint32_t j = tl.start + threadIdx.x, g = wp.slot_off + j;
  d.tgt[g] = -1;
  d.act[g] = 0;
  d.sampled[g] = 255;
  if (j < wp.n_init) {
    const uint32_t cell = (uint32_t)(d.cellkeys[wp.cell_off + j] & 0xFFFFFFFFull);   // ranked by placement
    d.flags[g] = kAlive;
    d.pos[g] = (int)cell;
    d.occ[wp.cell_off + cell] = (int)j;
    d.facing[g] = (uint8_t)(draw32(wp, j, 0u, ST_FACING) >> 30);
    d.energy[g] = wp.e_init;
    d.age[g] = 0;
    if (d.ep) {
      d.water[g] = d.ep[tl.world].w_init;
      d.biomass[g] = d.ep[tl.world].b_init;
      d.hp[g] = d.ep[tl.world].hp_max;
    }
    d.uid[g] = j;
    d.puid[g] = ~0ull;
  } else {
    d.flags[g] = 0;
    d.trait[g] = 0.0;
  }
}

// Initial weights of a list of (world, local slot) pairs, one block per entry
// (persistent).  list == nullptr: every slot j < n_init of every world, with
// entries enumerated through the per-world init counts.
template <int WDT>
__global__ __launch_bounds__(256) void k_emit_list(Dev d, Layout L, const uint32_t* __restrict__ list, uint32_t n,
                                                   int mode, double std1, double std2, double std3) {
  __shared__ uint32_t s_amax[128 + 128 + 16];
  __shared__ double s_red[4];
  __shared__ double2 tab[kTrigTable];
  load_trig(d.trig, tab);
  for (uint32_t e = blockIdx.x; e < n; e += gridDim.x) {
    const uint32_t w = list[2 * e], j = list[2 * e + 1];
    const WorldParams wp = d.wp[w];
    const uint32_t g = wp.slot_off + j;
    emit_agent<WDT>(d, L, wp, g, mode, j, std1, std2, std3, tab, s_amax, s_red);
    __syncthreads();
  }
}

// Parity mode: mark every slot "not evaluated" before the policy kernel runs.
__global__ __launch_bounds__(256) void k_prestep_fill(Dev d) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.total_slots) return;
  d.sampled[i] = 255;
  if (d.keep_logits) {
    const float nan = __builtin_nanf("");
    for (uint32_t a = 0; a < d.lgs; ++a) d.logits[(uint64_t)i * d.lgs + a] = nan;
  }
}

// Streaming-read probe (measurement only): every 16-byte block of p read once,
// grid-stride, 8 non-temporal loads in flight per lane; the XOR of the data
// goes to *sink only if it equals a constant, so the loads cannot be dropped.
typedef unsigned int probe_u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(512) void k_stream_read(const probe_u32x4* __restrict__ p, uint64_t n, uint32_t* sink) {
  constexpr int U = 8;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    probe_u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(p + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < n; i += stride) {
    const probe_u32x4 v = __builtin_nontemporal_load(p + i);
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x9E3779B9u) *sink = acc;
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free step (eco_world_step_static): the tile
// partials, birth lists and step counters of one object live in this array
// instead of the object's own buffers.  Each GPU the library runs on holds one
// copy until the process ends; every call on that GPU shares it.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// This GPU's address of the array (the array's name in host code is only a host
// stand-in): looked up once per device, with that device current, and kept.
hipError_t static_scratch(void** ptr, size_t* bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex lock;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(lock);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kStaticScratchBytes;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Host-side launchers (used by eco_runtime.cpp)
// ---------------------------------------------------------------------------
#define ECO_CHECK_LAUNCH() return hipGetLastError()

hipError_t launch_move(hipStream_t s, const Dev& d, const TileScratch& ts) {
  if (ts.n_slot_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_move, dim3(ts.n_slot_tiles), dim3(kSlotTile), 0, s, d, ts.slot_tiles, ts.part_slot);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_birth_claim_regrow(hipStream_t s, const Dev& d, const TileScratch& ts, uint32_t A) {
  const uint32_t nb = ts.n_slot_tiles + ts.n_cell_tiles;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_birth_claim_regrow, dim3(nb), dim3(256), 0, s, d, ts, A);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_birth_rank(hipStream_t s, const Dev& d, const TileScratch& ts) {
  hipLaunchKernelGGL(k_birth_rank_count, dim3(ts.n_slot_tiles), dim3(kSlotTile), 0, s, d, ts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_birth_rank_write, dim3(ts.n_slot_tiles), dim3(kSlotTile), 0, s, d, ts);
  ECO_CHECK_LAUNCH();
}
// Resident blocks per CU of the birth-commit kernel for this layout (its register
// and LDS use), so that the persistent grid is exactly one wave of resident blocks.
template <int WDT>
const void* birth_commit_fn(uint32_t H) {
  if (H == 32) return reinterpret_cast<const void*>(&k_birth_commit<WDT, 32>);
  if (H == 64) return reinterpret_cast<const void*>(&k_birth_commit<WDT, 64>);
  return reinterpret_cast<const void*>(&k_birth_commit<WDT, 128>);
}
hipError_t birth_commit_blocks_per_cu(const Layout& L, int* blocks) {
  const void* f = L.wdtype == 0 ? birth_commit_fn<0>(L.H1) : (L.wdtype == 1 ? birth_commit_fn<1>(L.H1)
                                                                              : birth_commit_fn<2>(L.H1));
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, f, 256, 0);
}

template <int WDT>
void launch_birth_commit_w(hipStream_t s, const Dev& d, const Layout& L, uint32_t blocks) {
  if (L.H1 == 32) hipLaunchKernelGGL((k_birth_commit<WDT, 32>), dim3(blocks), dim3(256), 0, s, d, L);
  else if (L.H1 == 64) hipLaunchKernelGGL((k_birth_commit<WDT, 64>), dim3(blocks), dim3(256), 0, s, d, L);
  else hipLaunchKernelGGL((k_birth_commit<WDT, 128>), dim3(blocks), dim3(256), 0, s, d, L);
}
hipError_t launch_step_small(hipStream_t s, const Dev& d, const Layout& L) {
  if (L.H1 != L.H2 || (L.H1 != 32 && L.H1 != 64 && L.H1 != 128)) return hipErrorInvalidValue;
#define ECO_SMALL(WW, E)                                                                                          \
  if (L.H1 == 32) hipLaunchKernelGGL((k_step_small<WW, 32, E>), dim3(1), dim3(1024), 0, s, d, L, L.A);           \
  else if (L.H1 == 64) hipLaunchKernelGGL((k_step_small<WW, 64, E>), dim3(1), dim3(1024), 0, s, d, L, L.A);      \
  else hipLaunchKernelGGL((k_step_small<WW, 128, E>), dim3(1), dim3(1024), 0, s, d, L, L.A);
  if (d.ep) {
    if (L.wdtype == 0) { ECO_SMALL(0, true) }
    else if (L.wdtype == 1) { ECO_SMALL(1, true) }
    else { ECO_SMALL(2, true) }
  } else {
    if (L.wdtype == 0) { ECO_SMALL(0, false) }
    else if (L.wdtype == 1) { ECO_SMALL(1, false) }
    else { ECO_SMALL(2, false) }
  }
#undef ECO_SMALL
  ECO_CHECK_LAUNCH();
}
hipError_t launch_birth_commit(hipStream_t s, const Dev& d, const Layout& L, uint32_t blocks) {
  if (L.H1 != L.H2 || (L.H1 != 32 && L.H1 != 64 && L.H1 != 128)) return hipErrorInvalidValue;
  if (L.wdtype == 0) launch_birth_commit_w<0>(s, d, L, blocks);
  else if (L.wdtype == 1) launch_birth_commit_w<1>(s, d, L, blocks);
  else launch_birth_commit_w<2>(s, d, L, blocks);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_compact(hipStream_t s, const Dev& d, const TileScratch& ts, int init, int only_world) {
  hipLaunchKernelGGL(k_compact_count, dim3(ts.n_slot_tiles), dim3(kSlotTile), 0, s, d, ts, only_world);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_compact_write, dim3(ts.n_slot_tiles + ts.n_cell_tiles), dim3(kSlotTile), 0, s, d, ts, init,
                     only_world);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_stream_read(hipStream_t s, const void* p, uint64_t n16, uint32_t* sink, uint32_t blocks,
                              uint32_t threads) {
  hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(threads), 0, s, reinterpret_cast<const probe_u32x4*>(p), n16,
                     sink);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_prestep_fill(hipStream_t s, const Dev& d) {
  hipLaunchKernelGGL(k_prestep_fill, dim3((d.total_slots + 255) / 256), dim3(256), 0, s, d);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_flowdir(hipStream_t s, const Dev& d, const TileScratch& ts, int world) {
  if (ts.n_cell_tiles == 0 || !d.rock) return hipSuccess;
  hipLaunchKernelGGL(k_flowdir, dim3(ts.n_cell_tiles), dim3(256), 0, s, d, ts.cell_tiles, world);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_render(hipStream_t s, const Dev& d, const TileScratch& ts, int world) {
  if (ts.n_cell_tiles == 0 || !d.rgb) return hipSuccess;
  hipLaunchKernelGGL(k_render, dim3(ts.n_cell_tiles), dim3(256), 0, s, d, ts.cell_tiles, world);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_resource_total(hipStream_t s, const Dev& d, int only_world) {
  hipLaunchKernelGGL(k_resource_total, dim3(d.n_worlds), dim3(kScanThreads), 0, s, d, only_world);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_init_cells(hipStream_t s, const Dev& d, const Tile* tiles, uint32_t nt) {
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_cells, dim3(nt), dim3(256), 0, s, d, tiles);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_placement(hipStream_t s, const Dev& d, const Tile* cell_tiles, uint32_t nt, const void* pinfo,
                            uint32_t* cnt, uint32_t* start) {
  if (nt == 0) return hipSuccess;
  const PlaceInfo* pi = reinterpret_cast<const PlaceInfo*>(pinfo);
  hipLaunchKernelGGL(k_place_count, dim3(nt), dim3(256), 0, s, d, cell_tiles, pi, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_place_scan, dim3(d.n_worlds), dim3(kScanThreads), 0, s, pi, cnt, start);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_place_scatter, dim3(nt), dim3(256), 0, s, d, cell_tiles, pi, cnt, start);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_place_rank, dim3(nt), dim3(256), 0, s, d, cell_tiles, pi, start);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_init_agents(hipStream_t s, const Dev& d, const Tile* tiles, uint32_t nt) {
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_agents, dim3(nt), dim3(kSlotTile), 0, s, d, tiles);
  ECO_CHECK_LAUNCH();
}
hipError_t launch_emit_list(hipStream_t s, const Dev& d, const Layout& L, const uint32_t* list, uint32_t n, int mode,
                            double std1, double std2, double std3, uint32_t blocks) {
  if (n == 0) return hipSuccess;
  if (L.wdtype == 0)
    hipLaunchKernelGGL(k_emit_list<0>, dim3(blocks), dim3(256), 0, s, d, L, list, n, mode, std1, std2, std3);
  else if (L.wdtype == 1)
    hipLaunchKernelGGL(k_emit_list<1>, dim3(blocks), dim3(256), 0, s, d, L, list, n, mode, std1, std2, std3);
  else
    hipLaunchKernelGGL(k_emit_list<2>, dim3(blocks), dim3(256), 0, s, d, L, list, n, mode, std1, std2, std3);
  ECO_CHECK_LAUNCH();
}

}  // namespace eco
