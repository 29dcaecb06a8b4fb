// eco_forward.hip -- policy step of every live agent (observation, MLP, sample, turn/claim).
//
// One wavefront evaluates one agent at a time; each agent's weights are read
// exactly once per step (no reuse across agents), so the kernel is bound by HBM
// bandwidth, not by the matrix cores: the product is a batched GEMV with a
// private matrix per agent (Sec. 3.3 per-agent policies).
//
// Per agent:
//  1. Observation (Sec. 3.2 "Sensors", App. F "Around" layout): the S x S
//     window around the agent, rotated so the agent faces the top row, four
//     channels per cell (agent present, resource, wall, occupant energy bin),
//     then the scalar sensors (energy, age, resource here, reproduction
//     eligibility, and the 4-way compass when n_s = 8).  Written to LDS.  The
//     four channels of a cell come from its sense byte, built for the step by
//     a per-cell pass before this kernel.
//  2. h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), l = W3 h2 + b3 (Sec. 3.3).
//     The weights of a layer are stored as 16-byte blocks [k-block][row]; lane
//     l streams block it*64+l, so every load instruction of the wave reads one
//     contiguous kilobyte, and each lane owns whole output rows (no cross-lane
//     reduction in layers 1-2).  The input values come from LDS as broadcasts.
//  3. Softmax sample with a Philox uniform (Sec. 3.3), temperature 1.
//  4. Turns; a FORWARD mover whose target was empty at step start claims it
//     with atomicMin on the slot id (lowest slot wins, Sec. 3.2 "Actions").
#include "eco_device.h"

#ifndef ECO_FWD_WDT
#error "compile with -DECO_FWD_WDT=0|1|2"
#endif

namespace eco {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int WDT>
struct WTraits;
template <>
struct WTraits<0> { static constexpr int VPL = 4; };
template <>
struct WTraits<1> { static constexpr int VPL = 8; };
template <>
struct WTraits<2> { static constexpr int VPL = 16; };

__device__ __forceinline__ float bf16lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// acc += sum over the VPL values of one 16-byte weight block times xs[0..VPL),
// in ascending value order.
template <int WDT>
__device__ __forceinline__ float dot_block(u32x4 w, const float* __restrict__ xs, float acc);

template <>
__device__ __forceinline__ float dot_block<0>(u32x4 w, const float* __restrict__ xs, float acc) {
  const float4 x = *reinterpret_cast<const float4*>(xs);
  acc = __builtin_fmaf(__uint_as_float(w.x), x.x, acc);
  acc = __builtin_fmaf(__uint_as_float(w.y), x.y, acc);
  acc = __builtin_fmaf(__uint_as_float(w.z), x.z, acc);
  acc = __builtin_fmaf(__uint_as_float(w.w), x.w, acc);
  return acc;
}

template <>
__device__ __forceinline__ float dot_block<1>(u32x4 w, const float* __restrict__ xs, float acc) {
  const float4 a = *reinterpret_cast<const float4*>(xs);
  const float4 b = *reinterpret_cast<const float4*>(xs + 4);
  acc = __builtin_fmaf(bf16lo(w.x), a.x, acc);
  acc = __builtin_fmaf(bf16hi(w.x), a.y, acc);
  acc = __builtin_fmaf(bf16lo(w.y), a.z, acc);
  acc = __builtin_fmaf(bf16hi(w.y), a.w, acc);
  acc = __builtin_fmaf(bf16lo(w.z), b.x, acc);
  acc = __builtin_fmaf(bf16hi(w.z), b.y, acc);
  acc = __builtin_fmaf(bf16lo(w.w), b.z, acc);
  acc = __builtin_fmaf(bf16hi(w.w), b.w, acc);
  return acc;
}

// FP8 E4M3 (OCP) pairs decoded by the gfx950 conversion instruction.
__device__ __forceinline__ float dot_fp8_word(uint32_t w, float4 x, float acc) {
  const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
  const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
  acc = __builtin_fmaf(lo[0], x.x, acc);
  acc = __builtin_fmaf(lo[1], x.y, acc);
  acc = __builtin_fmaf(hi[0], x.z, acc);
  acc = __builtin_fmaf(hi[1], x.w, acc);
  return acc;
}

template <>
__device__ __forceinline__ float dot_block<2>(u32x4 w, const float* __restrict__ xs, float acc) {
  acc = dot_fp8_word(w.x, *reinterpret_cast<const float4*>(xs), acc);
  acc = dot_fp8_word(w.y, *reinterpret_cast<const float4*>(xs + 4), acc);
  acc = dot_fp8_word(w.z, *reinterpret_cast<const float4*>(xs + 8), acc);
  acc = dot_fp8_word(w.w, *reinterpret_cast<const float4*>(xs + 12), acc);
  return acc;
}

// One layer of one agent as a stream of 16-byte blocks stored [KB][ROWS]: lane l
// reads block it*64 + l of iteration it, so each load instruction of the wave
// reads one contiguous kilobyte.  ROWS = 64: row l, k-block it.  ROWS = 32: row
// l%32, k-block 2it + l/32 (the two half-waves are summed afterwards).  ROWS =
// 128: row l + 64 (it%2), k-block it/2 (two accumulators).
struct Seg {
  const u32x4* blk;   // the layer's first block
  int nblk;           // KB * ROWS blocks
  int nit;            // ceil(nblk / 64) iterations
};

template <int ROWS>
__device__ __forceinline__ Seg make_seg(const uint8_t* __restrict__ wbase, uint32_t off, int KB) {
  Seg s;
  s.blk = reinterpret_cast<const u32x4*>(wbase + off);
  s.nblk = KB * ROWS;
  s.nit = (s.nblk + 63) >> 6;
  return s;
}

// The lane's block of iteration it.  With 32 rows an odd KB leaves the upper
// half-wave of the last iteration past the layer: it re-reads the layer's last
// block (that value is never used), so every load stays inside the layer.
template <int ROWS>
__device__ __forceinline__ u32x4 ld_block(const Seg& s, int it, int lane) {
  int e = it * 64 + lane;
  if (ROWS == 32) e = min(e, s.nblk - 1);
  return __builtin_nontemporal_load(s.blk + e);
}

// acc += the products of block w of iteration it (u: it modulo the ring length,
// which is even, so u % 2 == it % 2).  Accumulation order per row is fixed by
// (ROWS, KB) only, never by the ring length.
template <int WDT, int ROWS>
__device__ __forceinline__ void consume_block(const u32x4& w, int it, int u, int KB, const float* __restrict__ xs,
                                              int lane, float (&acc)[ROWS == 128 ? 2 : 1]) {
  constexpr int VPL = WTraits<WDT>::VPL;
  if (ROWS == 64) {
    acc[0] = dot_block<WDT>(w, xs + it * VPL, acc[0]);
  } else if (ROWS == 32) {
    const int kb = 2 * it + (lane >> 5);
    if (kb < KB) acc[0] = dot_block<WDT>(w, xs + kb * VPL, acc[0]);
  } else {
    acc[u & 1] = dot_block<WDT>(w, xs + (it >> 1) * VPL, acc[u & 1]);
  }
}

// Streams segment `cur` through a ring of U registers holding loads in flight.
// The segment's iterations are taken in chunks of U (the last chunk padded): on
// entry w[u] holds (or is loading) iteration u of cur; each block consumed is
// replaced at once by the load of the iteration U further on, so the wave keeps
// U loads in flight without draining between chunks, and the last chunk's
// slots take iterations 0..U-1 of the next segment (the agent's second layer,
// or the next agent's first layer), so the stream does not drain between layers
// or agents either.  Padding iterations, and the next segment when there is
// none, re-read the segment's last block (a cache hit, never used), so that
// every slot issues exactly one load per chunk and no load sits in a branch.
template <int WDT, int ROWS, int U>
__device__ __forceinline__ void stream_seg(u32x4 (&w)[U], const Seg& cur, int KB, const float* __restrict__ xs,
                                           int lane, float (&acc)[ROWS == 128 ? 2 : 1], const Seg& nxt,
                                           bool has_nxt) {
  static_assert(U % 2 == 0, "U must be even");
  const int nit = cur.nit;
  const int last = ((nit - 1) / U) * U;   // first iteration of the last chunk
  int it0 = 0;
  for (; it0 < last; it0 += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      consume_block<WDT, ROWS>(w[u], it0 + u, u, KB, xs, lane, acc);
      w[u] = ld_block<ROWS>(cur, min(it0 + U + u, nit - 1), lane);
      // keeps the scheduler from unpacking blocks ahead of their turn, which
      // doubles the registers a block holds and, at two waves per SIMD, spills
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  const Seg& t = has_nxt ? nxt : cur;
  const int tl = has_nxt ? 0 : nit - 1;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (it0 + u < nit) consume_block<WDT, ROWS>(w[u], it0 + u, u, KB, xs, lane, acc);
    w[u] = ld_block<ROWS>(t, has_nxt ? min(u, t.nit - 1) : tl, lane);
  }
}

// The first blocks of a segment into an empty ring.
template <int ROWS, int U>
__device__ __forceinline__ void ring_start(u32x4 (&w)[U], const Seg& s, int lane) {
#pragma unroll
  for (int u = 0; u < U; ++u) w[u] = ld_block<ROWS>(s, min(u, s.nit - 1), lane);
}

// A field of the kernel's by-value Dev argument, read from the kernel's argument
// segment where it is used.  The argument segment holds the kernel's explicit
// arguments in order, each at its natural alignment, so Dev (the first) starts
// at offset 0.  The segment pointer passes through an empty asm statement first,
// which the compiler cannot see through: each use is one scalar load from the
// scalar cache, instead of a value hoisted to the kernel's entry and held in a
// scalar register across the agent loop (the policy kernel reads some thirty
// such pointers, more than the scalar registers hold, and the excess spilled).
template <typename T>
__device__ __forceinline__ T dev_arg(uint32_t offset) {
  typedef const __attribute__((address_space(4))) uint8_t* seg_ptr;
  seg_ptr p = (seg_ptr)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return *(const __attribute__((address_space(4))) T*)(p + offset);
}
#define DEV_ARG(field) dev_arg<decltype(Dev::field)>(offsetof(Dev, field))
// The same for the Layout argument, which follows Dev at Layout's alignment.
constexpr uint32_t kLayoutArg = (sizeof(Dev) + alignof(Layout) - 1) / alignof(Layout) * alignof(Layout);
#define LAYOUT_ARG(field) dev_arg<decltype(Layout::field)>(kLayoutArg + offsetof(Layout, field))

// Biases (BF16 for BF16 storage, FP32 otherwise) and FP8 row scales of one
// agent, loaded as raw words when the agent starts and converted where they are
// used, so no layer epilogue waits for memory.
template <int WDT>
__device__ __forceinline__ uint32_t load_bias_raw(const uint8_t* __restrict__ p, int i) {
  if (WDT == 1) return reinterpret_cast<const uint16_t*>(p)[i];
  return reinterpret_cast<const uint32_t*>(p)[i];
}
template <int WDT>
__device__ __forceinline__ float bias_of(uint32_t raw) {
  return (WDT == 1) ? __uint_as_float(raw << 16) : __uint_as_float(raw);
}
template <int WDT>
__device__ __forceinline__ float scale_of(uint32_t raw) {
  return (WDT == 2) ? __uint_as_float(raw) : 1.0f;
}

template <int WDT, int H>
struct Tail {
  static constexpr int RPL = (H == 128) ? 2 : 1;
  uint32_t b1[RPL], b2[RPL], s1[RPL], s2[RPL], b3, s3;
};

template <int WDT, int H>
__device__ __forceinline__ void load_tail(const uint8_t* __restrict__ wbase, const Layout& L, int lane,
                                          Tail<WDT, H>& t) {
#pragma unroll
  for (int r = 0; r < Tail<WDT, H>::RPL; ++r) {
    const int j = (H == 32) ? (lane & 31) : lane + 64 * r;
    t.b1[r] = load_bias_raw<WDT>(wbase + LAYOUT_ARG(s_b1), j);
    t.b2[r] = load_bias_raw<WDT>(wbase + LAYOUT_ARG(s_b2), j);
    t.s1[r] = (WDT == 2) ? reinterpret_cast<const uint32_t*>(wbase + LAYOUT_ARG(s_sc1))[j] : 0u;
    t.s2[r] = (WDT == 2) ? reinterpret_cast<const uint32_t*>(wbase + LAYOUT_ARG(s_sc2))[j] : 0u;
  }
  t.b3 = load_bias_raw<WDT>(wbase + LAYOUT_ARG(s_b3), lane >> 3);
  t.s3 = (WDT == 2) ? reinterpret_cast<const uint32_t*>(wbase + LAYOUT_ARG(s_sc3))[lane >> 3] : 0u;
}

// Epilogue of one hidden layer: half-wave combine, scale, bias, ReLU, result to
// LDS hs[0..ROWS).
template <int WDT, int ROWS>
__device__ __forceinline__ void layer_epilogue(float (&acc)[ROWS == 128 ? 2 : 1], float* __restrict__ hs, int lane,
                                               const uint32_t (&bias)[ROWS == 128 ? 2 : 1],
                                               const uint32_t (&scale)[ROWS == 128 ? 2 : 1]) {
  if (ROWS == 32) acc[0] += __shfl_xor(acc[0], 32);
#pragma unroll
  for (int r = 0; r < (ROWS == 128 ? 2 : 1); ++r) {
    const int j = (ROWS == 32) ? (lane & 31) : lane + 64 * r;
    float v = acc[r];
    if (WDT == 2) v *= scale_of<WDT>(scale[r]);
    v += bias_of<WDT>(bias[r]);
    v = fmaxf(v, 0.0f);
    if (ROWS != 32 || lane < 32) hs[j] = v;
  }
  wave_sync();
}

// Output layer [8][H2] values: lane l = 8a + g sums H2/8 products of row a,
// then a butterfly over g; logit a (rows a >= A are zero).  The lane's weight
// words are loaded before layer 2 streams (load_w3) and used after it.
template <int WDT, int H2>
struct W3 {
  static constexpr int NV = H2 / 8;                                      // values per lane
  static constexpr int NW = (WDT == 0) ? NV : (WDT == 1) ? NV / 2 : NV / 4;  // 32-bit words per lane
  uint32_t w[NW];
};

template <int WDT, int H2>
__device__ __forceinline__ void load_w3(const uint8_t* __restrict__ wbase, const Layout& L, int lane, W3<WDT, H2>& o) {
  constexpr int NV = W3<WDT, H2>::NV, NW = W3<WDT, H2>::NW;
  constexpr int VB = (WDT == 0) ? 4 : (WDT == 1) ? 2 : 1;  // bytes per value
  const int first = (lane >> 3) * H2 + (lane & 7) * NV;
  const uint8_t* p = wbase + LAYOUT_ARG(s_w3) + (uint64_t)first * VB;  // 4 * NW bytes, aligned to min(16, 4 * NW)
  if (NW >= 4) {
#pragma unroll
    for (int q = 0; q < NW / 4; ++q) {
      const u32x4 v = reinterpret_cast<const u32x4*>(p)[q];
      o.w[4 * q] = v.x;
      o.w[4 * q + 1] = v.y;
      o.w[4 * q + 2] = v.z;
      o.w[4 * q + 3] = v.w;
    }
  } else if (NW == 2) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    o.w[0] = v.x;
    o.w[NW - 1] = v.y;
  } else {
    o.w[0] = *reinterpret_cast<const uint32_t*>(p);
  }
}

template <int WDT, int H2>
__device__ __forceinline__ float output_layer(const W3<WDT, H2>& o, const float* __restrict__ h2, int lane,
                                              uint32_t b3, uint32_t s3) {
  constexpr int NV = W3<WDT, H2>::NV;
  const float* hv = h2 + (lane & 7) * NV;
  float part = 0.0f;
  if (WDT == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) part = __builtin_fmaf(__uint_as_float(o.w[q]), hv[q], part);
  } else if (WDT == 1) {
#pragma unroll
    for (int q = 0; q < NV / 2; ++q) {
      part = __builtin_fmaf(bf16lo(o.w[q]), hv[2 * q + 0], part);
      part = __builtin_fmaf(bf16hi(o.w[q]), hv[2 * q + 1], part);
    }
  } else {
#pragma unroll
    for (int q = 0; q < NV / 4; ++q)
      part = dot_fp8_word(o.w[q], make_float4(hv[4 * q], hv[4 * q + 1], hv[4 * q + 2], hv[4 * q + 3]), part);
  }
  part += __shfl_xor(part, 1);
  part += __shfl_xor(part, 2);
  part += __shfl_xor(part, 4);
  if (WDT == 2) part *= scale_of<WDT>(s3);
  part += bias_of<WDT>(b3);
  return part;
}

// The ninth output row (the ecology's attack logit).  Its raw weights (lane l
// takes h2 entries l, and l + 64 when H2 = 128; lanes >= 32 idle when H2 = 32),
// bias and FP8 scale are loaded with the output layer's, before layer 2 streams;
// after it, a sum over the whole wave, which every lane returns.
template <int WDT, int H2>
struct Row9 {
  uint32_t w[H2 == 128 ? 2 : 1];
  uint32_t b, s, t;   // t: bias slot 9, the log temperature of a nine-action head
};

template <int WDT, int H2>
__device__ __forceinline__ void load_row9(const uint8_t* __restrict__ wbase, const Layout& L, int lane,
                                          Row9<WDT, H2>& o) {
#pragma unroll
  for (int r = 0; r < (H2 == 128 ? 2 : 1); ++r) {
    const uint32_t e = 8u * H2 + (uint32_t)(lane + 64 * r);   // element of row 8
    if (H2 == 32 && lane >= 32) o.w[r] = 0u;
    else if (WDT == 0) o.w[r] = reinterpret_cast<const uint32_t*>(wbase + LAYOUT_ARG(s_w3))[e];
    else if (WDT == 1) o.w[r] = reinterpret_cast<const uint16_t*>(wbase + LAYOUT_ARG(s_w3))[e];
    else o.w[r] = (wbase + LAYOUT_ARG(s_w3))[e];
  }
  o.b = load_bias_raw<WDT>(wbase + LAYOUT_ARG(s_b3), 8);
  o.s = (WDT == 2) ? reinterpret_cast<const uint32_t*>(wbase + LAYOUT_ARG(s_sc3))[8] : 0u;
  o.t = (LAYOUT_ARG(temp) && LAYOUT_ARG(A) > 8) ? load_bias_raw<WDT>(wbase + LAYOUT_ARG(s_b3), 9) : 0u;
}

template <int WDT, int H2>
__device__ __forceinline__ float ninth_logit(const Row9<WDT, H2>& o, const float* __restrict__ h2, int lane) {
  float part = 0.0f;
#pragma unroll
  for (int r = 0; r < (H2 == 128 ? 2 : 1); ++r) {
    const int j = (H2 == 32) ? (lane & 31) : lane + 64 * r;
    const float v = (WDT == 0) ? __uint_as_float(o.w[r])
                    : (WDT == 1) ? bf16lo(o.w[r])
                                 : __builtin_amdgcn_cvt_pk_f32_fp8(o.w[r], false)[0];
    part = __builtin_fmaf(v, h2[j], part);   // lanes >= 32 of H2 = 32 hold a zero weight
  }
#pragma unroll
  for (int dd = 1; dd < 64; dd <<= 1) part += __shfl_xor(part, dd);
  if (WDT == 2) part *= scale_of<WDT>(o.s);
  return part + bias_of<WDT>(o.b);
}

// Exclusive prefix of the per-world live counts into off[0..n] (wave 0 of the block).
__device__ __forceinline__ void world_offsets(const WorldVar* __restrict__ wv, uint32_t n, uint32_t* off) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    const uint32_t per = (n + 63) / 64;
    const uint32_t lo = tid * per, hi = min(lo + per, n);
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; ++i) s += wv[i].n_live;
    uint32_t inc = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t v = __shfl_up(inc, d);
      if (tid >= d) inc += v;
    }
    uint32_t run = inc - s;
    for (uint32_t i = lo; i < hi; ++i) {
      off[i] = run;
      run += wv[i].n_live;
    }
    if (tid == 63) off[n] = inc;
  }
  __syncthreads();
}

// Wave-uniform loads through the scalar cache.  None of these words is written by
// this kernel before the agent they belong to is processed (turns write only the
// processed agent's facing byte), so the scalar cache cannot return a stale value.
template <typename T>
__device__ __forceinline__ T sload(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Uniform description of one agent of the wave's chunk (with its world's grid;
// the world's other parameters are read where they are used).
struct AgentCtx {
  uint32_t w, local, slot, step;
  int pos, facing, energy, age;
  uint32_t W, H, cell_off;
};

// Field of world w's parameters, read from the scalar cache where it is used.
template <typename T>
__device__ __forceinline__ T world_param(uint32_t w, uint32_t offset) {
  return sload(reinterpret_cast<const T*>(reinterpret_cast<const uint8_t*>(DEV_ARG(wp) + w) + offset));
}
#define WORLD_PARAM(w, field) world_param<decltype(WorldParams::field)>(w, offsetof(WorldParams, field))

// Agent g of the step's live list (woff in LDS: exclusive world offsets); w is a
// world index not past g's world.
__device__ __forceinline__ AgentCtx load_agent(const uint32_t* woff, uint32_t g, uint32_t w) {
  while (g >= uni(woff[w + 1])) ++w;
  AgentCtx c;
  c.w = w;
  const uint32_t slot_off = WORLD_PARAM(w, slot_off);
  c.W = WORLD_PARAM(w, W);
  c.H = WORLD_PARAM(w, H);
  c.cell_off = WORLD_PARAM(w, cell_off);
  c.local = (uint32_t)sload(DEV_ARG(live) + slot_off + (g - uni(woff[w])));
  c.slot = slot_off + c.local;
  c.step = (uint32_t)sload(&DEV_ARG(wv)[w].step);
  c.pos = sload(DEV_ARG(pos) + c.slot);
  c.energy = sload(DEV_ARG(energy) + c.slot);
  c.age = sload(DEV_ARG(age) + c.slot);
  const uint32_t fw = sload(reinterpret_cast<const uint32_t*>(DEV_ARG(facing) + (c.slot & ~3u)));
  c.facing = (int)((fw >> (8 * (c.slot & 3u))) & 0xFFu);
  return c;
}

constexpr int kMaxWindowCellsPerLane = 4;  // S <= 15: S*S <= 256 cells over 64 lanes
constexpr int kEcoLane = 58;               // lanes 58..63 of the last window slot: cells 250..255, never in a window

// Sense bytes (or, with colour vision, rendered words) of agent c's window (Sec.
// 3.2 sensors, App. F layout): lane owns window cells lane + 64k, row r = i / S
// counted from the far front, column from the agent's left; the window is
// rotated so the agent faces row 0.  Row 0 lies L.ahead0 cells ahead: R for the
// "Around" layout (the agent in the middle), S - 1 for "Front" (the agent in the
// middle of the last row, nothing behind it seen).
// WORDS: the window is read as 4-byte words (colour vision or the ecology), else
// as sense bytes; a compile-time choice, so the byte path carries none of the
// word path's code.
template <bool WORDS>
__device__ __forceinline__ void gather_sense(const Layout& L, const AgentCtx& c, int lane,
                                             uint32_t (&sv)[kMaxWindowCellsPerLane]) {
  const AgentCtx& wp = c;   // the world's grid
  const int S = (int)LAYOUT_ARG(S), R = (int)LAYOUT_ARG(R), SS = S * S;
  const int ax = c.pos % (int)wp.W, ay = c.pos / (int)wp.W;
  const int dx = dir_dx(c.facing), dy = dir_dy(c.facing), rx = -dy, ry = dx;
#pragma unroll
  for (int k = 0; k < kMaxWindowCellsPerLane; ++k) {
    const int i = lane + 64 * k;
    sv[k] = 0;
    if (i < SS) {
      const int r = i / S, col = i - r * S;
      const int fw = (int)LAYOUT_ARG(ahead0) - r, rt = col - R;
      int cx = ax + fw * dx + rt * rx, cy = ay + fw * dy + rt * ry;
      if (cx < 0) cx += (int)wp.W; else if (cx >= (int)wp.W) cx -= (int)wp.W;
      if (cy < 0) cy += (int)wp.H; else if (cy >= (int)wp.H) cy -= (int)wp.H;
      const uint32_t cell = wp.cell_off + (uint32_t)cy * wp.W + (uint32_t)cx;
      if constexpr (WORDS) sv[k] = DEV_ARG(rgb)[cell];
      else sv[k] = DEV_ARG(sense)[cell];
    } else if (WORDS && k == kMaxWindowCellsPerLane - 1 && LAYOUT_ARG(ecology) && lane >= kEcoLane) {
      // ecology: the own cell's water, energy, biomass and the agent's water,
      // biomass, health ride in window slots no window reaches (S*S <= 225 < 250),
      // fetched with the window
      const int j = lane - kEcoLane;
      const int32_t* src = j == 0 ? DEV_ARG(cw) : j == 1 ? DEV_ARG(ce) : j == 2 ? DEV_ARG(cb)
                           : j == 3 ? DEV_ARG(water) : j == 4 ? DEV_ARG(biomass) : DEV_ARG(hp);
      sv[k] = (uint32_t)src[j < 3 ? wp.cell_off + (uint32_t)c.pos : c.slot];
    }
  }
}

// Window word of cell i (uniform) from the lane that gathered it.
__device__ __forceinline__ uint32_t window_word(const uint32_t (&sv)[kMaxWindowCellsPerLane], int i) {
  const int k = i >> 6;
  const uint32_t v = k == 0 ? sv[0] : (k == 1 ? sv[1] : (k == 2 ? sv[2] : sv[3]));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, i & 63);
}

// Observation of agent c into LDS xs[0..D): four channels per window cell, then
// the scalars (energy, age, resource here, eligibility, compass when n_s = 8).
// Cell channels: agent, resource, wall, energy bin from the sense byte; with
// colour vision the rendered R, G, B (8-bit values times 2^-8) and the
// elevation difference, zero on the flat torus.
template <bool WORDS>
__device__ __forceinline__ void write_observation(const Layout& L, const AgentCtx& c, int lane,
                                                  const uint32_t (&sv)[kMaxWindowCellsPerLane], float* xs) {
  const int SS = (int)(LAYOUT_ARG(S) * LAYOUT_ARG(S));
  const int centre = (int)(LAYOUT_ARG(ahead0) * LAYOUT_ARG(S) + LAYOUT_ARG(R));  // the agent's own cell
  // colour words carry the cell's sense bits and rock height in their top byte
  const uint32_t here = (WORDS && LAYOUT_ARG(colour)) ? window_word(sv, centre) : 0u;
  const int own_rock = (int)(here >> 27);
#pragma unroll
  for (int k = 0; k < kMaxWindowCellsPerLane; ++k) {
    const int i = lane + 64 * k;
    if (i < SS) {
      const uint32_t v = sv[k];
      float4 o;
      if constexpr (!WORDS) {
        o = make_float4((float)(v & 1u), (float)((v >> 1) & 1u), (float)((v >> 2) & 1u), (float)(v >> 3));
      } else if (LAYOUT_ARG(colour)) {   // rendered colour; the elevation difference from the rock bits (0 without terrain)
        o = make_float4(ldexpf((float)(v & 0xFFu), -8), ldexpf((float)((v >> 8) & 0xFFu), -8),
                        ldexpf((float)((v >> 16) & 0xFFu), -8), ldexpf((float)((int)(v >> 27) - own_rock), -3));
      } else {   // ecology: agent present, then the water, energy, biomass levels
        o = make_float4((float)((v >> 24) & 1u), ldexpf((float)(v & 0xFFu), -4), ldexpf((float)((v >> 8) & 0xFFu), -4),
                        ldexpf((float)((v >> 16) & 0xFFu), -4));
      }
      reinterpret_cast<float4*>(xs)[i] = o;
    } else if (WORDS && k == kMaxWindowCellsPerLane - 1 && LAYOUT_ARG(ecology) && lane >= kEcoLane) {
      // fetched into this unused window slot: the own cell's levels (external
      // sensor, min(units, 255) * 2^-4) and the agent's water, biomass, health
      const int j = lane - kEcoLane, u = (int)sv[k];
      if (j < 3) xs[4 * SS + 5 + j] = ldexpf((float)min(u, 255), -4);
      else xs[4 * SS + 2 + (j - 3)] = ldexpf((float)u, j == 3 ? -8 : (j == 4 ? -3 : -7));
    }
  }
  const float res_here = (float)((here >> 25) & 1u);

  wave_sync();
  if (WORDS && LAYOUT_ARG(ecology)) {
    // internal: energy, age (here), water, biomass, health (written above by the
    // lanes that fetched them); external: the own cell's levels (written above);
    // the compass when n_s = 12
    if (lane < 2) xs[4 * SS + lane] = lane == 0 ? ldexpf((float)c.energy, -8) : ldexpf((float)min(c.age, 1024), -10);
    else if (lane >= 8 && lane < (int)LAYOUT_ARG(ns)) xs[4 * SS + lane] = (lane - 8 == c.facing) ? 1.0f : 0.0f;
  } else if (lane < (int)LAYOUT_ARG(ns)) {
    float v;
    if (lane == 0) v = ldexpf((float)c.energy, -8);
    else if (lane == 1) v = ldexpf((float)min(c.age, 1024), -10);
    else if (lane == 2) v = (WORDS && LAYOUT_ARG(colour)) ? res_here : xs[4 * centre + 1];  // resource here: the own cell's resource
    else if (lane == 3) v = (c.energy >= WORLD_PARAM(c.w, e_repro)) ? 1.0f : 0.0f;
    else v = (lane - 4 == c.facing) ? 1.0f : 0.0f;
    xs[4 * SS + lane] = v;
  }
  wave_sync();
}

// At least three waves per SIMD (two for the 8- and 16-deep rings of the word
// path, whose loads in flight need the registers): the compiler's own register
// choice moves between these variants from build to build, and a wave fewer
// costs more than the few registers it frees.
template <int H, int U, bool WORDS>
constexpr int kMinWavesPerSimd = (U == 16 || (WORDS && U == 8)) ? 2 : 3;

// NINE: a ninth output row (the ecology with attack: a ninth action; with the
// evolving temperature and eight actions: the log temperature), from
// ninth_logit; a separate instantiation, so that the other kernels carry none of
// its code.
template <int WDT, int H, int U, bool WORDS, bool NINE>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(kMinWavesPerSimd<H, U, WORDS>)))
void k_forward(Dev d, Layout L) {
  constexpr int VPL = WTraits<WDT>::VPL;
  extern __shared__ __align__(16) float smem[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  uint32_t* woff = reinterpret_cast<uint32_t*>(smem);
  const uint32_t woff_words = (d.n_worlds + 1 + 3) & ~3u;
  float* xs = smem + woff_words + wave * (L.Dpad + 2 * 128);
  float* h1s = xs + L.Dpad;
  float* h2s = h1s + 128;

  for (uint32_t i = L.D + lane; i < L.Dpad; i += 64) xs[i] = 0.0f;  // padding stays zero
  world_offsets(d.wv, d.n_worlds, woff);
  const uint32_t total = woff[d.n_worlds];
  const uint32_t n_waves = gridDim.x * wpb;
  const uint32_t gw = blockIdx.x * wpb + wave;
  const uint32_t chunk = (total + n_waves - 1) / n_waves;
  const uint32_t g_lo = gw * chunk, g_hi = min(g_lo + chunk, total);
  if (g_lo >= g_hi) return;

  static_assert(WORDS || !NINE, "a ninth action needs the ecology's window words");
  constexpr int NA = NINE ? 9 : 8;   // the most actions this instantiation samples from

  AgentCtx cur = load_agent(woff, g_lo, find_world(woff, d.n_worlds, g_lo));
  uint32_t sv[kMaxWindowCellsPerLane];
  gather_sense<WORDS>(L, cur, lane, sv);
  const int KB2 = (int)L.H1 / VPL;   // layer-2 k-blocks (H1 == H; a run-time value, so the compiler keeps the stream a loop)
  // the weight stream: layer 1 and layer 2 of each agent in turn, U blocks in flight
  u32x4 ring[U];
  ring_start<H, U>(ring, make_seg<H>(d.store + (uint64_t)cur.slot * L.sstride, L.s_w1, (int)L.KBv), lane);
  for (uint32_t g = g_lo; g < g_hi; ++g) {
    const AgentCtx& wp = cur;   // the world's grid
    // Window cell ahead of the agent (row ahead0 - 1, column R), when the window has
    // one: the move claim reads its agent and wall channels from the observation
    // (with colour vision, from the sense bits of its rendered word).
    const uint32_t ahead0 = LAYOUT_ARG(ahead0);
    const int front = (ahead0 >= 1) ? (int)((ahead0 - 1) * LAYOUT_ARG(S) + LAYOUT_ARG(R)) : -1;
    // ---- 1. observation into LDS (window bytes fetched one agent ahead) ----
    write_observation<WORDS>(L, cur, lane, sv, xs);
    const uint32_t front_word = (WORDS && front >= 0) ? window_word(sv, front) : 0u;
    // the next agent's context and window bytes, in flight while this agent streams
    const bool has_next = g + 1 < g_hi;
    AgentCtx nxt = cur;
    uint32_t sn[kMaxWindowCellsPerLane];
    if (has_next) {
      nxt = load_agent(woff, g + 1, cur.w);
      gather_sense<WORDS>(L, nxt, lane, sn);
    }

    // ---- 2. the agent's MLP, weights streamed once from HBM ----
    const uint8_t* wbase = DEV_ARG(store) + (uint64_t)cur.slot * LAYOUT_ARG(sstride);
    Tail<WDT, H> tl;
    load_tail<WDT, H>(wbase, L, lane, tl);
    const Seg s1 = make_seg<H>(wbase, LAYOUT_ARG(s_w1), (int)L.KBv), s2 = make_seg<H>(wbase, LAYOUT_ARG(s_w2), KB2);
    float acc1[H == 128 ? 2 : 1] = {};
    stream_seg<WDT, H, U>(ring, s1, (int)L.KBv, xs, lane, acc1, s2, true);
    layer_epilogue<WDT, H>(acc1, h1s, lane, tl.b1, tl.s1);
    W3<WDT, H> w3;
    load_w3<WDT, H>(wbase, L, lane, w3);
    Row9<WDT, H> r9;
    if (NINE) load_row9<WDT, H>(wbase, L, lane, r9);
    const Seg n1 = make_seg<H>(DEV_ARG(store) + (uint64_t)nxt.slot * LAYOUT_ARG(sstride), LAYOUT_ARG(s_w1), (int)L.KBv);
    float acc2[H == 128 ? 2 : 1] = {};
    stream_seg<WDT, H, U>(ring, s2, KB2, h1s, lane, acc2, n1, has_next);
    layer_epilogue<WDT, H>(acc2, h2s, lane, tl.b2, tl.s2);
    const float lg = output_layer<WDT, H>(w3, h2s, lane, tl.b3, tl.s3);
    const float l8 = NINE ? ninth_logit<WDT, H>(r9, h2s, lane) : 0.0f;

    // ---- 3. softmax inverse-CDF sample ----
    const int A = (int)LAYOUT_ARG(A);
    float l[9];
#pragma unroll
    for (int a = 0; a < 8; ++a) l[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lg), 8 * a));
    l[8] = l8;
    float m = l[0];
#pragma unroll
    for (int a = 1; a < NA; ++a)
      if (a < A) m = fmaxf(m, l[a]);
    // one exponential per lane (lane 8a + g holds logit a), then gathered in order.
    // An evolving temperature tau = exp(theta_T) divides the logits; theta_T is the
    // stored parameter after the output biases, so logit A (a zero weight row plus
    // that bias slot) equals it: one of the eight logits, the ninth one (the
    // ecology's eight actions), or bias slot 9 itself (its nine).  The largest
    // logits weigh exactly 1.
    float e_lane, inv_tau = 1.0f;
    const bool temp = LAYOUT_ARG(temp) != 0;
    if (temp) {
      float lt = 0.0f;
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (a == A) lt = l[a];
      if (NINE) lt = (A == 8) ? l8 : bias_of<WDT>(r9.t);
      inv_tau = expf(-lt);
      const float x = lg - m;
      e_lane = ((lane >> 3) < A) ? (x == 0.0f ? 1.0f : expf(x * inv_tau)) : 0.0f;
    } else {
      e_lane = ((lane >> 3) < A) ? expf(lg - m) : 0.0f;
    }
    float C[9], wk[9], accum = 0.0f;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      wk[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(e_lane), 8 * a));
      accum += wk[a];
      C[a] = accum;
    }
    if (NINE) {   // the ninth action's weight (zero when logit 8 is the log temperature)
      const float x8 = l8 - m;
      wk[8] = (A > 8) ? (temp ? (x8 == 0.0f ? 1.0f : expf(x8 * inv_tau)) : expf(x8)) : 0.0f;
      C[8] = accum + wk[8];
    }
    const uint32_t x0 = philox10(cur.local, cur.step, ST_ACTION, 0u, WORLD_PARAM(cur.w, key0), WORLD_PARAM(cur.w, key1)).x;
    const float u = (float)(x0 >> 8) * 0x1p-24f;
    const float t = u * C[NA - 1];   // = C[A - 1]: the weights of actions >= A are zero
    int as = -1;
#pragma unroll
    for (int a = 0; a < NA; ++a)
      if (as < 0 && a < A && t < C[a]) as = a;
    if (as < 0) {
#pragma unroll
      for (int a = 0; a < NA; ++a)
        if (a < A && wk[a] > 0.0f) as = a;
    }

    // ---- 4. bookkeeping, turn, move claim (lane 0) ----
    const uint32_t slot = cur.slot;
    constexpr uint32_t lgs = NINE ? 16u : 8u;   // the logit buffer's stride (Dev::lgs)
    if (DEV_ARG(keep_logits) && (lane & 7) == 0) DEV_ARG(logits)[(uint64_t)slot * lgs + (lane >> 3)] = ((lane >> 3) < A) ? lg : 0.0f;
    if (NINE && DEV_ARG(keep_logits) && lane == 0) DEV_ARG(logits)[(uint64_t)slot * lgs + 8] = l8;
    if (lane == 0 && DEV_ARG(dry)) DEV_ARG(sampled)[slot] = (uint8_t)as;
    if (lane == 0 && !DEV_ARG(dry)) {
      const int a = DEV_ARG(inject) ? (int)DEV_ARG(act_in)[slot] : as;
      const int f = cur.facing;
      DEV_ARG(sampled)[slot] = (uint8_t)as;
      DEV_ARG(act)[slot] = (uint8_t)a;
      int tg = -1;
      if (a == TURN_L) DEV_ARG(facing)[slot] = (uint8_t)((f + 3) & 3);
      else if (a == TURN_R) DEV_ARG(facing)[slot] = (uint8_t)((f + 1) & 3);
      else if (a == FORWARD) {
        const uint32_t tc = neighbour(wp, (uint32_t)cur.pos, f, +1);
        bool free_cell;
        if (WORDS && front >= 0) {  // agent and wall bits of the window word
          free_cell = ((front_word >> 24) & 5u) == 0u;
        } else if (front >= 0) {  // the observation holds the cell ahead as seen at step start
          free_cell = xs[4 * front] == 0.0f && xs[4 * front + 2] == 0.0f;
        } else {
          free_cell = DEV_ARG(occ)[wp.cell_off + tc] == -1 &&
                      !(WORLD_PARAM(cur.w, has_walls) && DEV_ARG(wall)[wp.cell_off + tc]);
        }
        if (free_cell) {
          atomicMin(&DEV_ARG(claim)[wp.cell_off + tc], slot);
          tg = (int)tc;
        }
      }
      DEV_ARG(tgt)[slot] = tg;
    }
    // An attacker (it neither turns nor moves) stamps the 3x3 square directly
    // ahead of it, rows 1..3 ahead, one column to either side, with this step;
    // the move kernel kills whoever stands on a stamped cell after the moves.
    // The square can wrap onto the attacker's own cell on a small torus: that
    // cell is skipped.  Equal stamps from several attackers are idempotent.  In
    // the ecology (whose attack is the ninth action) the strikes are counted
    // instead, each costing health, and an attacker strikes each distinct cell
    // once: lane (ahead, side) is cell (ahead mod Lf, side mod Lr) of the square,
    // Lf and Lr the torus lengths along and across the facing, so it repeats an
    // earlier lane exactly when side + 1 >= Lr or ahead > Lf (sides below 3).
    if (WORLD_PARAM(cur.w, attack) && !DEV_ARG(dry)) {
      const int a = DEV_ARG(inject) ? (int)DEV_ARG(act_in)[slot] : as;
      if (a == (NINE ? (int)ATTACK_ECO : (int)ATTACK) && lane < 9) {
        const int ahead = 1 + lane / 3, side = lane % 3 - 1;
        const uint32_t c = offset_cell(wp, (uint32_t)cur.pos, cur.facing, ahead, side);
        bool skip = c == (uint32_t)cur.pos;
        if (NINE) {
          const int lf = (cur.facing & 1) ? (int)wp.W : (int)wp.H, lr = (cur.facing & 1) ? (int)wp.H : (int)wp.W;
          skip |= side + 1 >= lr || ahead > lf;
        }
        if (!skip) {
          if (NINE) atomicAdd(&DEV_ARG(mark)[wp.cell_off + c], 1u);
          else DEV_ARG(mark)[wp.cell_off + c] = cur.step + 1u;
        }
      }
    }
    if (has_next) {
      cur = nxt;
#pragma unroll
      for (int k = 0; k < kMaxWindowCellsPerLane; ++k) sv[k] = sn[k];
    }
  }
}

}  // namespace eco

// Host-side launcher for this storage type: picks the (H, U) instantiation.
namespace eco {
#define ECO_CAT2(a, b) a##b
#define ECO_CAT(a, b) ECO_CAT2(a, b)
hipError_t ECO_CAT(launch_forward_w, ECO_FWD_WDT)(int H, int U, dim3 grid, dim3 block, size_t shmem,
                                                  hipStream_t s, const Dev& d, const Layout& L) {
  const bool words = (L.colour | L.ecology) != 0, nine = L.A + L.temp > 8;
#define ECO_CASE(HH, UU)                                                                                  \
  if (H == HH && U == UU) {                                                                               \
    if (nine) hipLaunchKernelGGL((k_forward<ECO_FWD_WDT, HH, UU, true, true>), grid, block, shmem, s, d, L);  \
    else if (words) hipLaunchKernelGGL((k_forward<ECO_FWD_WDT, HH, UU, true, false>), grid, block, shmem, s, d, L); \
    else hipLaunchKernelGGL((k_forward<ECO_FWD_WDT, HH, UU, false, false>), grid, block, shmem, s, d, L);     \
    return hipGetLastError();                                                                             \
  }
  ECO_CASE(32, 4) ECO_CASE(32, 8) ECO_CASE(32, 16)
  ECO_CASE(64, 4) ECO_CASE(64, 8) ECO_CASE(64, 16)
  ECO_CASE(128, 4) ECO_CASE(128, 8) ECO_CASE(128, 16)
#undef ECO_CASE
  return hipErrorInvalidValue;
}
// The kernel a launch of this storage type with (H, U) runs (graph nodes name it);
// mode 0: sense bytes, 1: window words, 2: window words and a ninth action.
const void* ECO_CAT(forward_kernel_w, ECO_FWD_WDT)(int H, int U, int mode) {
#define ECO_FN(HH, UU)                                                                                \
  if (H == HH && U == UU)                                                                             \
    return mode == 2 ? reinterpret_cast<const void*>(&k_forward<ECO_FWD_WDT, HH, UU, true, true>)      \
           : mode == 1 ? reinterpret_cast<const void*>(&k_forward<ECO_FWD_WDT, HH, UU, true, false>)   \
                       : reinterpret_cast<const void*>(&k_forward<ECO_FWD_WDT, HH, UU, false, false>);
  ECO_FN(32, 4) ECO_FN(32, 8) ECO_FN(32, 16)
  ECO_FN(64, 4) ECO_FN(64, 8) ECO_FN(64, 16)
  ECO_FN(128, 4) ECO_FN(128, 8) ECO_FN(128, 16)
#undef ECO_FN
  return nullptr;
}
}  // namespace eco
