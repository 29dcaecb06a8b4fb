// eco_runtime.cpp -- host side of libeco: the C ABI of include/eco.h.
//
// Owns the device buffers of one or more worlds, runs the deterministic init,
// sequences the step kernels on the caller's stream (eagerly, or as a replayed
// hipGraph), and implements the parity / checkpoint hooks.  Compiled by hipcc
// as HIP host code; all step arithmetic lives in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "eco_device.h"

namespace eco {
hipError_t launch_forward_w0(int H, int U, dim3 grid, dim3 block, size_t shmem, hipStream_t s, const Dev& d,
                             const Layout& L);
hipError_t launch_forward_w1(int H, int U, dim3 grid, dim3 block, size_t shmem, hipStream_t s, const Dev& d,
                             const Layout& L);
const void* forward_kernel_w0(int H, int U, int mode);
const void* forward_kernel_w1(int H, int U, int mode);
const void* forward_kernel_w2(int H, int U, int mode);
hipError_t launch_forward_w2(int H, int U, dim3 grid, dim3 block, size_t shmem, hipStream_t s, const Dev& d,
                             const Layout& L);
hipError_t launch_move(hipStream_t s, const Dev& d, const TileScratch& ts);
hipError_t launch_birth_claim_regrow(hipStream_t s, const Dev& d, const TileScratch& ts, uint32_t A);
hipError_t launch_birth_rank(hipStream_t s, const Dev& d, const TileScratch& ts);
hipError_t launch_birth_commit(hipStream_t s, const Dev& d, const Layout& L, uint32_t blocks);
hipError_t launch_step_small(hipStream_t s, const Dev& d, const Layout& L);
hipError_t birth_commit_blocks_per_cu(const Layout& L, int* blocks);
hipError_t static_scratch(void** ptr, size_t* bytes);
hipError_t launch_compact(hipStream_t s, const Dev& d, const TileScratch& ts, int init, int only_world);
hipError_t launch_prestep_fill(hipStream_t s, const Dev& d);
hipError_t launch_stream_read(hipStream_t s, const void* p, uint64_t n16, uint32_t* sink, uint32_t blocks,
                              uint32_t threads);
hipError_t launch_resource_total(hipStream_t s, const Dev& d, int only_world);
hipError_t launch_render(hipStream_t s, const Dev& d, const TileScratch& ts, int world);
hipError_t launch_flowdir(hipStream_t s, const Dev& d, const TileScratch& ts, int world);
hipError_t launch_init_cells(hipStream_t s, const Dev& d, const Tile* tiles, uint32_t nt);
hipError_t launch_init_agents(hipStream_t s, const Dev& d, const Tile* tiles, uint32_t nt);
hipError_t launch_emit_list(hipStream_t s, const Dev& d, const Layout& L, const uint32_t* list, uint32_t n, int mode,
                            double std1, double std2, double std3, uint32_t blocks);
hipError_t launch_placement(hipStream_t s, const Dev& d, const Tile* cell_tiles, uint32_t nt, const void* pinfo,
                            uint32_t* cnt, uint32_t* start);
}  // namespace eco

using namespace eco;

namespace {

constexpr uint32_t kSlotTileH = 256;
constexpr uint32_t kCellTileH = 1024;
constexpr uint32_t kSlotPartH = 16;
constexpr uint32_t kCellPartH = 4;
constexpr uint32_t kMaxWorldsH = 1024;
enum { EMIT_INIT = 0, EMIT_REQUANT = 2 };

thread_local std::string g_err;

eco_status fail(eco_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

uint64_t round_up(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

uint64_t bern_threshold(float p) {
  double t = std::floor((double)p * 4294967296.0);
  if (t < 0) t = 0;
  if (t > 4294967296.0) t = 4294967296.0;
  return (uint64_t)t;
}

}  // namespace

struct eco_world {
  uint32_t n_worlds = 0;
  std::vector<eco_world_desc> descs;
  std::vector<WorldParams> wp;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  bool has_alloc = false;
  eco_allocator alloc{};
  std::vector<std::pair<void*, size_t>> allocations;
  Dev d{};
  Layout L{};
  double std1 = 0, std2 = 0, std3 = 0;
  uint32_t total_slots = 0, total_cells = 0;
  std::vector<Tile> slot_tiles_h, cell_tiles_h;
  std::vector<uint32_t> tile_rng_h;
  Tile* slot_tiles = nullptr;
  Tile* cell_tiles = nullptr;
  uint32_t n_slot_tiles = 0, n_cell_tiles = 0;
  uint32_t* part_slot = nullptr;
  unsigned long long* part_cell = nullptr;
  uint32_t* tile_rng = nullptr;
  TileScratch ts{};
  // placement (init): per-world bucket table {first bucket, key shift} (+ a sentinel),
  // bucket counts and starts
  void* place_info = nullptr;
  uint32_t* place_cnt = nullptr;
  uint32_t* place_start = nullptr;
  uint32_t n_buckets = 0;
  std::vector<uint32_t> place_info_h;
  uint32_t* emit_list = nullptr;
  int n_cus = 256;
  int birth_bpc = 4;        // resident birth-commit blocks per CU
  eco_launch launch{4, 4, 8, 0};
  uint32_t rt_flags = ECO_RT_USE_GRAPH;
  // Graphs of m whole steps (1 <= m <= kGraphSteps) replayed by eco_world_step
  // under ECO_RT_USE_GRAPH, kept per m (at most kGraphKeep of them): n steps run
  // as n / kGraphSteps replays of the kGraphSteps-step graph and one of the
  // remainder's, so consecutive steps are separated by a kernel boundary inside
  // a graph, not by a graph launch.
  struct StepGraph {
    uint32_t n = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<StepGraph> sgraphs;
  bool broken = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  size_t ev_used = 0;
  // Graphs of n whole steps with event-record nodes around every policy-kernel
  // launch (ECO_RT_TIME_KERNELS together with ECO_RT_USE_GRAPH), one per n used.
  struct TimedGraph {
    uint32_t n = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> events;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pairs;
  };
  std::vector<TimedGraph> tgraphs;
  eco_kernel_times kt{};
  uint64_t device_bytes = 0;
};

namespace {

eco_status dev_fail(eco_world* w, hipError_t e, const char* what) {
  w->broken = true;
  return fail(ECO_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(w, call, what)                       \
  do {                                              \
    hipError_t e_ = (call);                         \
    if (e_ != hipSuccess) return dev_fail(w, e_, what); \
  } while (0)

void* dalloc(eco_world* w, size_t bytes) {
  if (bytes == 0) bytes = 16;
  void* p = nullptr;
  if (w->has_alloc) {
    p = w->alloc.alloc(bytes, w->alloc.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p) {
    w->allocations.push_back({p, bytes});
    w->device_bytes += bytes;
  }
  return p;
}

void free_all(eco_world* w) {
  for (auto& a : w->allocations) {
    if (w->has_alloc) w->alloc.free(a.first, w->alloc.ctx);
    else (void)hipFree(a.first);
  }
  w->allocations.clear();
}

eco_status check_desc(const eco_world_desc& d, uint32_t i) {
  char buf[160];
  auto bad = [&](eco_status st, const char* field, const char* why) {
    snprintf(buf, sizeof buf, "world %u: %s %s", i, field, why);
    return fail(st, buf);
  };
  if (d.struct_size != sizeof(eco_world_desc)) return bad(ECO_EINVAL, "struct_size", "!= sizeof(eco_world_desc)");
  if (d.width < 1 || d.height < 1) return bad(ECO_EINVAL, "width/height", "must be >= 1");
  if ((uint64_t)d.width * d.height >= (1ull << 31)) return bad(ECO_EINVAL, "width*height", "must be < 2^31");
  if (d.capacity < 1) return bad(ECO_EINVAL, "capacity", "must be >= 1");
  if (d.n_agents_init > d.capacity) return bad(ECO_EINVAL, "n_agents_init", "exceeds capacity");
  if ((uint64_t)d.n_agents_init > (uint64_t)d.width * d.height) return bad(ECO_EINVAL, "n_agents_init", "exceeds cells");
  if (d.window < 1 || d.window % 2 == 0) return bad(ECO_EINVAL, "window", "must be odd");
  if (d.window > d.width || d.window > d.height) return bad(ECO_EINVAL, "window", "larger than the grid");
  if (d.window > 15) return bad(ECO_ENOTSUP, "window", "above 15 has no policy kernel");
  if ((d.flags & ECO_DESC_ECOLOGY) ? (d.n_scalars != 8 && d.n_scalars != 12) : (d.n_scalars != 4 && d.n_scalars != 8))
    return bad(ECO_EINVAL, "n_scalars", "must be 4 or 8 (8 or 12 in the ecology)");
  if (d.n_actions != 5 && d.n_actions != 7 && d.n_actions != 8 && d.n_actions != 9)
    return bad(ECO_EINVAL, "n_actions", "must be 5 or 7 (8, or 9 with attack, in the ecology)");
  if (d.e_repro <= 0) return bad(ECO_EINVAL, "e_repro", "must be > 0");
  if (d.wdtype > ECO_W_FP8E4M3) return bad(ECO_EINVAL, "wdtype", "unknown");
  if (!(d.resource_density >= 0.0f && d.resource_density <= 1.0f)) return bad(ECO_EINVAL, "resource_density", "outside [0,1]");
  if (!(d.regrow_prob >= 0.0f && d.regrow_prob <= 1.0f)) return bad(ECO_EINVAL, "regrow_prob", "outside [0,1]");
  if (!(d.mutation_sigma >= 0.0f) || std::isinf(d.mutation_sigma)) return bad(ECO_EINVAL, "mutation_sigma", "must be finite and >= 0");
  if (d.attack_enabled > 1) return bad(ECO_EINVAL, "attack_enabled", "must be 0 or 1");
  if (d.attack_enabled && d.n_actions != ((d.flags & ECO_DESC_ECOLOGY) ? 9u : 7u))
    return bad(ECO_EINVAL, "attack_enabled", "needs n_actions = 7 (9 in the ecology)");
  if (d.flags & ~(ECO_DESC_FRONT_VISION | ECO_DESC_EVOLVE_TEMPERATURE | ECO_DESC_COLOUR_VISION | ECO_DESC_ECOLOGY |
                  ECO_DESC_TERRAIN))
    return bad(ECO_EINVAL, "flags", "has unknown bits");
  if (d.flags & ECO_DESC_ECOLOGY) {
    const eco_ecology& e = d.eco;
    if (d.n_actions != (d.attack_enabled ? 9u : 8u))
      return bad(ECO_EINVAL, "n_actions", "must be 8 in the ecology (9 with attack)");
    if (e.attack_damage < 0 || e.attack_damage > (1 << 20))
      return bad(ECO_EINVAL, "eco.attack_damage", "outside [0, 2^20]");
    if ((d.flags & ECO_DESC_TERRAIN) && (e.terrain_scale < 1 || e.sea_level < 0 || e.sea_level > 32 ||
                                         e.water_per_depth < 0))
      return bad(ECO_EINVAL, "eco.terrain_*", "terrain_scale >= 1, sea_level in [0, 32], water_per_depth >= 0");
    if (e.hp_max <= 0 || e.hp_child <= 0 || e.hp_child > e.hp_max) return bad(ECO_EINVAL, "eco.hp_*", "bad limits");
    if (e.age_shift < 0 || e.age_shift > 31) return bad(ECO_EINVAL, "eco.age_shift", "outside [0, 31]");
    if (e.cap_water < 0 || e.cap_energy < 0 || e.cap_biomass < 0 || e.eat_water < 0 || e.eat_biomass < 0 ||
        e.w_cost < 0 || e.e_cost_move < 0 || e.hp_overspend < 0 || e.hp_heal < 0 || e.heal_energy < 0 ||
        e.w_init < 0 || e.b_init < 0 || e.w_child < 0 || e.b_child < 0 || e.b_repro < e.b_child ||
        e.water_site < 0 || e.energy_site < 0 || e.biomass_site < 0 || e.cell_energy_max < 0 || d.e_eat < 0 ||
        d.e_cost < 0 || d.e_child < 0)
      return bad(ECO_EINVAL, "eco", "amounts must be >= 0 and b_repro >= b_child");
    auto unit = [](float p) { return p >= 0.0f && p <= 1.0f; };
    if (!(e.photo_rate >= 0.0f) || std::isinf(e.photo_rate) || !unit(e.water_density) || !unit(e.energy_density) ||
        !unit(e.biomass_density))
      return bad(ECO_EINVAL, "eco", "densities must lie in [0,1] and photo_rate be finite and >= 0");
  } else if (d.n_actions >= 8) {
    return bad(ECO_EINVAL, "n_actions", "8 or 9 needs ECO_DESC_ECOLOGY");
  }
  if ((d.flags & ECO_DESC_TERRAIN) && !(d.flags & ECO_DESC_ECOLOGY))
    return bad(ECO_EINVAL, "flags", "terrain needs ECO_DESC_ECOLOGY");
  auto okh = [](uint32_t h) { return h == 32 || h == 64 || h == 128; };
  if (!okh(d.hidden1) || !okh(d.hidden2)) return bad(ECO_ENOTSUP, "hidden1/hidden2", "must be 32, 64 or 128");
  if (d.hidden1 != d.hidden2) return bad(ECO_ENOTSUP, "hidden1/hidden2", "must be equal");
  return ECO_OK;
}

// Device layout of one agent's parameters (see eco_device.h).
void make_layout(const eco_world_desc& d, Layout& L, double& s1, double& s2, double& s3) {
  L = Layout{};
  L.S = d.window;
  L.R = (d.window - 1) / 2;
  L.ns = d.n_scalars;
  L.D = 4 * d.window * d.window + d.n_scalars;
  L.H1 = d.hidden1;
  L.H2 = d.hidden2;
  L.A = d.n_actions;
  L.wdtype = d.wdtype;
  L.ahead0 = (d.flags & ECO_DESC_FRONT_VISION) ? d.window - 1 : L.R;
  L.temp = (d.flags & ECO_DESC_EVOLVE_TEMPERATURE) ? 1u : 0u;
  L.colour = (d.flags & ECO_DESC_COLOUR_VISION) ? 1u : 0u;
  L.ecology = (d.flags & ECO_DESC_ECOLOGY) ? 1u : 0u;
  L.R3 = (L.A + L.temp > 8) ? 16u : 8u;   // output rows and bias slots, the log temperature included
  L.P = L.D * L.H1 + L.H1 + L.H1 * L.H2 + L.H2 + L.H2 * L.A + L.A + L.temp;
  L.p_w1 = 0;
  L.p_b1 = L.p_w1 + L.H1 * L.D;
  L.p_w2 = L.p_b1 + L.H1;
  L.p_b2 = L.p_w2 + L.H2 * L.H1;
  L.p_w3 = L.p_b2 + L.H2;
  L.p_b3 = L.p_w3 + L.A * L.H2;
  L.KB1 = L.D / 4;
  L.u_w1 = 0;
  L.u_b1 = L.KB1 * L.H1;
  L.u_w2 = L.u_b1 + L.H1 / 4;
  L.u_b2 = L.u_w2 + (L.H1 / 4) * L.H2;
  L.u_w3 = L.u_b2 + L.H2 / 4;
  L.u_b3 = L.u_w3 + L.R3 * (L.H2 / 4);
  L.u_end = L.u_b3 + L.R3 / 4;
  const uint32_t vpl = d.wdtype == ECO_W_FP32 ? 4 : (d.wdtype == ECO_W_BF16 ? 8 : 16);
  L.KBv = (L.D + vpl - 1) / vpl;
  L.Dpad = L.KBv * vpl;
  uint64_t o = 0;
  auto put = [&](uint32_t& field, uint64_t bytes) {
    field = (uint32_t)o;
    o = round_up(o + bytes, 16);
  };
  if (d.wdtype == ECO_W_FP32) {
    put(L.s_w1, (uint64_t)L.KBv * L.H1 * 16);
    put(L.s_b1, 4ull * L.H1);
    put(L.s_w2, (uint64_t)(L.H1 / 4) * L.H2 * 16);
    put(L.s_b2, 4ull * L.H2);
    put(L.s_w3, 4ull * L.R3 * L.H2);
    put(L.s_b3, 4ull * L.R3);
  } else if (d.wdtype == ECO_W_BF16) {
    put(L.s_w1, (uint64_t)L.KBv * L.H1 * 16);
    put(L.s_b1, 2ull * L.H1);
    put(L.s_w2, (uint64_t)(L.H1 / 8) * L.H2 * 16);
    put(L.s_b2, 2ull * L.H2);
    put(L.s_w3, 2ull * L.R3 * L.H2);
    put(L.s_b3, 2ull * L.R3);
  } else {
    put(L.s_w1, (uint64_t)L.KBv * L.H1 * 16);
    put(L.s_w2, (uint64_t)(L.H1 / 16) * L.H2 * 16);
    put(L.s_w3, 1ull * L.R3 * L.H2);
    put(L.s_b1, 4ull * L.H1);
    put(L.s_b2, 4ull * L.H2);
    put(L.s_b3, 4ull * L.R3);
    put(L.s_sc1, 4ull * L.H1);
    put(L.s_sc2, 4ull * L.H2);
    put(L.s_sc3, 4ull * L.R3);
  }
  L.sstride = round_up(o, 256);
  L.mstride = (d.wdtype == ECO_W_FP32) ? L.sstride : round_up(16ull * L.u_end, 256);
  s1 = std::sqrt(1.0 / (double)L.D);
  s2 = std::sqrt(1.0 / (double)L.H1);
  s3 = std::sqrt(1.0 / (double)L.H2);
}

// Bytes one forward pass of one agent reads from its weight block (algorithmic).
uint64_t weight_bytes(const Layout& L) {
  const uint64_t nw = (uint64_t)L.H1 * L.D + (uint64_t)L.H2 * L.H1 + (uint64_t)L.A * L.H2;
  const uint64_t nb = (uint64_t)L.H1 + L.H2 + L.A;
  if (L.wdtype == ECO_W_FP32) return 4 * (nw + nb);
  if (L.wdtype == ECO_W_BF16) return 2 * (nw + nb);
  return nw + 4 * nb + 4 * nb;  // FP8 weights, FP32 biases and row scales
}

// The Box-Muller angle table: cos and sin of 2 pi a / 256, a = 0..255.  The
// angle is reduced exactly by quarter turns and octant symmetry, so libm only
// sees arguments in [0, pi / 4] and the multiples of a quarter turn are exact.
std::vector<double2> angle_table() {
  std::vector<double2> t(kTrigTable);
  const int quarter = kTrigTable / 4;
  for (int a = 0; a < kTrigTable; ++a) {
    const int q = a / quarter, m = a % quarter;   // a = q quarter + m, m in [0, 64)
    double cb, sb;                                // cos, sin of 2 pi m / 256 in [0, pi / 2)
    if (2 * m <= quarter) {
      const double b = 2.0 * M_PI * (double)m / (double)kTrigTable;
      cb = std::cos(b);
      sb = std::sin(b);
    } else {                                      // pi / 2 - b = 2 pi (64 - m) / 256
      const double b = 2.0 * M_PI * (double)(quarter - m) / (double)kTrigTable;
      cb = std::sin(b);
      sb = std::cos(b);
    }
    const double c = q == 0 ? cb : (q == 1 ? -sb : (q == 2 ? -cb : sb));
    const double s = q == 0 ? sb : (q == 1 ? cb : (q == 2 ? -sb : -cb));
    t[a] = make_double2(c, s);
  }
  return t;
}

void upload_world_params(eco_world* w) {
  for (uint32_t i = 0; i < w->n_worlds; ++i) {
    w->wp[i].key0 = (uint32_t)(w->descs[i].seed & 0xFFFFFFFFu);
    w->wp[i].key1 = (uint32_t)(w->descs[i].seed >> 32);
  }
}

eco_status sync(eco_world* w) {
  HIPCHK(w, hipStreamSynchronize(w->stream), "hipStreamSynchronize");
  return ECO_OK;
}

uint32_t emit_blocks(eco_world* w) { return (uint32_t)std::max(1, w->n_cus * 4); }
// Birth commit: one 256-thread block per birth, persistent, as many blocks as
// can be resident at once (the kernel is bound by its noise arithmetic; more
// resident waves hide the parent reads, and a grid beyond residency would start
// its last blocks late and leave the chip idle behind them).
uint32_t birth_blocks(eco_world* w) { return (uint32_t)std::max(1, w->n_cus * w->birth_bpc); }

// Full deterministic init of every world.
eco_status run_init(eco_world* w) {
  hipStream_t s = w->stream;
  Dev& d = w->d;
  HIPCHK(w, hipMemcpyAsync((void*)d.wp, w->wp.data(), sizeof(WorldParams) * w->n_worlds, hipMemcpyHostToDevice, s),
         "upload world params");
  std::vector<WorldVar> wv(w->n_worlds);
  for (uint32_t i = 0; i < w->n_worlds; ++i) {
    wv[i] = WorldVar{};
    wv[i].uid_next = w->descs[i].n_agents_init;
  }
  HIPCHK(w, hipMemcpyAsync(d.wv, wv.data(), sizeof(WorldVar) * w->n_worlds, hipMemcpyHostToDevice, s), "upload vars");
  HIPCHK(w, hipMemsetAsync(d.flags, 0, w->total_slots, s), "clear flags");
  HIPCHK(w, hipMemsetAsync(d.ring, 0, sizeof(eco_stats) * kStatsRing * w->n_worlds, s), "clear stats");
  HIPCHK(w, launch_init_cells(s, d, w->cell_tiles, w->n_cell_tiles), "init cells");
  HIPCHK(w, launch_flowdir(s, d, w->ts, -1), "flow directions");
  HIPCHK(w, hipMemsetAsync(w->place_cnt, 0, 4ull * w->n_buckets, s), "clear placement counts");
  HIPCHK(w, launch_placement(s, d, w->cell_tiles, w->n_cell_tiles, w->place_info, w->place_cnt, w->place_start),
         "placement");
  HIPCHK(w, launch_init_agents(s, d, w->slot_tiles, w->n_slot_tiles), "init agents");
  std::vector<uint32_t> list;
  for (uint32_t i = 0; i < w->n_worlds; ++i)
    for (uint32_t j = 0; j < w->descs[i].n_agents_init; ++j) {
      list.push_back(i);
      list.push_back(j);
    }
  const uint32_t n = (uint32_t)(list.size() / 2);
  if (n) {
    HIPCHK(w, hipMemcpyAsync(w->emit_list, list.data(), list.size() * 4, hipMemcpyHostToDevice, s), "upload list");
    HIPCHK(w, launch_emit_list(s, d, w->L, w->emit_list, n, EMIT_INIT, w->std1, w->std2, w->std3, emit_blocks(w)),
           "init weights");
  }
  HIPCHK(w, launch_compact(s, d, w->ts, 1, -1), "compact");
  HIPCHK(w, launch_resource_total(s, d, -1), "resource total");
  eco_status st = sync(w);
  if (st != ECO_OK) return st;
  w->broken = false;
  return ECO_OK;
}

size_t forward_shmem(const eco_world* w, uint32_t wpb) {
  const uint32_t woff_words = (w->n_worlds + 1 + 3) & ~3u;
  return 4ull * (woff_words + (uint64_t)wpb * (w->L.Dpad + 256));
}

hipError_t launch_forward(eco_world* w, hipStream_t s, const Dev& d, const eco_launch& lc) {
  const dim3 grid((unsigned)std::max(1u, lc.blocks_per_cu * (uint32_t)w->n_cus));
  const dim3 block(64 * lc.waves_per_block);
  const size_t shmem = forward_shmem(w, lc.waves_per_block);
  if (w->L.wdtype == 0) return launch_forward_w0((int)w->L.H1, (int)lc.unroll, grid, block, shmem, s, d, w->L);
  if (w->L.wdtype == 1) return launch_forward_w1((int)w->L.H1, (int)lc.unroll, grid, block, shmem, s, d, w->L);
  return launch_forward_w2((int)w->L.H1, (int)lc.unroll, grid, block, shmem, s, d, w->L);
}

hipEvent_t take_event(eco_world* w) {
  if (w->ev_used == w->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    w->ev_pool.push_back(e);
  }
  return w->ev_pool[w->ev_used++];
}

// Kernel groups of one step, in order (each id names one timed group).
// (The sense bytes the policy kernel reads are built by the previous step's
// compaction launch, or by init and state writes.)
constexpr int kStepGroups[] = {ECO_K_FORWARD,    ECO_K_MOVE,         ECO_K_BIRTH_CLAIM,
                               ECO_K_BIRTH_SCAN, ECO_K_BIRTH_COMMIT, ECO_K_COMPACT};
const char* group_name(int k) {
  switch (k) {
    case ECO_K_FORWARD: return "forward kernel";
    case ECO_K_MOVE: return "move kernel";
    case ECO_K_BIRTH_CLAIM: return "birth claim / regrowth kernel";
    case ECO_K_BIRTH_SCAN: return "birth ranking kernels";
    case ECO_K_BIRTH_COMMIT: return "birth commit kernel";
    default: return "compaction kernels";
  }
}
hipError_t launch_group(eco_world* w, hipStream_t s, const Dev& d, const TileScratch& ts, int k) {
  switch (k) {
    case ECO_K_FORWARD: return launch_forward(w, s, d, w->launch);
    case ECO_K_MOVE: return launch_move(s, d, ts);
    case ECO_K_BIRTH_CLAIM: return launch_birth_claim_regrow(s, d, ts, w->L.A);
    case ECO_K_BIRTH_SCAN: return launch_birth_rank(s, d, ts);
    case ECO_K_BIRTH_COMMIT: return launch_birth_commit(s, d, w->L, birth_blocks(w));
    default: return launch_compact(s, d, ts, 0, -1);
  }
}

// An object of one small world steps with the policy kernel
// and one fused launch (k_step_small) unless ECO_RT_SPLIT_STEP asks for the
// separate kernels: its step is bound by launch latency, not by bytes.
constexpr uint32_t kSmallSlots = ECO_SMALL_STEP_MAX_SLOTS, kSmallCells = ECO_SMALL_STEP_MAX_CELLS;
bool small_step(const eco_world* w) {
  return w->n_worlds == 1 && w->total_slots <= kSmallSlots && w->total_cells <= kSmallCells &&
         !(w->rt_flags & ECO_RT_SPLIT_STEP);
}

// Enqueue one step's kernels.  timed: bracket each kernel group with events.
// ts: the tile partials the step's kernels use (the object's own, or the static
// array's for eco_world_step_static).
eco_status enqueue_step(eco_world* w, hipStream_t s, const Dev& d, const TileScratch& ts, bool timed) {
  if (d.keep_logits) HIPCHK(w, launch_prestep_fill(s, d), "prestep fill");
  if (small_step(w)) {   // the policy kernel, then the rest of the step in one launch (timed as MOVE)
    for (int k : {ECO_K_FORWARD, ECO_K_MOVE}) {
      hipEvent_t a = nullptr, b = nullptr;
      if (timed) {
        a = take_event(w);
        b = take_event(w);
        if (!a || !b) return dev_fail(w, hipErrorOutOfMemory, "timing events");
        HIPCHK(w, hipEventRecord(a, s), "event record");
      }
      if (k == ECO_K_FORWARD) HIPCHK(w, launch_forward(w, s, d, w->launch), "forward kernel");
      else HIPCHK(w, launch_step_small(s, d, w->L), "small-world step kernel");
      if (timed) {
        HIPCHK(w, hipEventRecord(b, s), "event record");
        w->ev_pending.push_back({k, {a, b}});
      }
    }
    return ECO_OK;
  }
  for (int k : kStepGroups) {
    hipEvent_t a = nullptr, b = nullptr;
    if (timed) {
      a = take_event(w);
      b = take_event(w);
      if (!a || !b) return dev_fail(w, hipErrorOutOfMemory, "timing events");
      HIPCHK(w, hipEventRecord(a, s), "event record");
    }
    HIPCHK(w, launch_group(w, s, d, ts, k), group_name(k));
    if (timed) {
      HIPCHK(w, hipEventRecord(b, s), "event record");
      w->ev_pending.push_back({k, {a, b}});
    }
  }
  return ECO_OK;
}

eco_status drain_events(eco_world* w) {
  if (w->ev_pending.empty()) return ECO_OK;
  HIPCHK(w, hipStreamSynchronize(w->stream), "hipStreamSynchronize");
  for (auto& p : w->ev_pending) {
    float ms = 0.0f;
    HIPCHK(w, hipEventElapsedTime(&ms, p.second.first, p.second.second), "hipEventElapsedTime");
    w->kt.ms[p.first] += ms;
    w->kt.launches[p.first] += 1;
  }
  w->ev_pending.clear();
  w->ev_used = 0;
  return ECO_OK;
}

void destroy_timed(eco_world::TimedGraph& t) {
  if (t.exec) (void)hipGraphExecDestroy(t.exec);
  if (t.graph) (void)hipGraphDestroy(t.graph);
  for (auto e : t.events) (void)hipEventDestroy(e);
  t = eco_world::TimedGraph{};
}

void destroy_step_graph(eco_world::StepGraph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = eco_world::StepGraph{};
}

// Drops every built graph (after the stream has drained: a replay may still run).
void drop_graph(eco_world* w) {
  if (w->sgraphs.empty() && w->tgraphs.empty()) return;
  (void)hipStreamSynchronize(w->stream);
  for (auto& g : w->sgraphs) destroy_step_graph(g);
  w->sgraphs.clear();
  for (auto& t : w->tgraphs) destroy_timed(t);
  w->tgraphs.clear();
}

constexpr uint32_t kGraphSteps = 32, kGraphKeep = 4;

// The graph of m whole steps (built and kept on first use).
eco_status step_graph(eco_world* w, uint32_t m, hipGraphExec_t* out) {
  for (auto& g : w->sgraphs)
    if (g.n == m) {
      *out = g.exec;
      return ECO_OK;
    }
  if (w->sgraphs.size() >= kGraphKeep) {
    (void)hipStreamSynchronize(w->stream);   // the oldest may still be replaying
    destroy_step_graph(w->sgraphs.front());
    w->sgraphs.erase(w->sgraphs.begin());
  }
  Dev d = w->d;
  d.inject = 0;
  d.dry = 0;
  d.keep_logits = (w->rt_flags & ECO_RT_KEEP_LOGITS) ? 1u : 0u;
  eco_world::StepGraph g;
  g.n = m;
  HIPCHK(w, hipStreamBeginCapture(w->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  eco_status st = ECO_OK;
  for (uint32_t i = 0; i < m && st == ECO_OK; ++i) st = enqueue_step(w, w->cap_stream, d, w->ts, false);
  const hipError_t e = hipStreamEndCapture(w->cap_stream, &g.graph);
  if (st != ECO_OK || e != hipSuccess) {
    destroy_step_graph(g);
    return st != ECO_OK ? st : dev_fail(w, e, "end capture");
  }
  const hipError_t ei = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    destroy_step_graph(g);
    return dev_fail(w, ei, "graph instantiate");
  }
  w->sgraphs.push_back(g);
  *out = g.exec;
  return ECO_OK;
}

// The untimed graphs that n steps replay: the kGraphSteps-step one and the remainder's.
eco_status prepare_step_graphs(eco_world* w, uint32_t n) {
  hipGraphExec_t ex = nullptr;
  eco_status st = ECO_OK;
  if (n >= kGraphSteps) st = step_graph(w, kGraphSteps, &ex);
  if (st == ECO_OK && n % kGraphSteps) st = step_graph(w, n % kGraphSteps, &ex);
  return st;
}

// Graph of n steps (captured like the step graphs) with an event-record node
// before and after every policy-kernel node, kept per n.  Only the dominant
// kernel is bracketed: each event node costs the replay several microseconds.
eco_status timed_graph(eco_world* w, uint32_t n, eco_world::TimedGraph** out) {
  for (auto& t : w->tgraphs)
    if (t.n == n) {
      *out = &t;
      return ECO_OK;
    }
  if (w->tgraphs.size() >= 4) {
    destroy_timed(w->tgraphs.front());
    w->tgraphs.erase(w->tgraphs.begin());
  }
  Dev d = w->d;
  d.inject = 0;
  d.dry = 0;
  d.keep_logits = (w->rt_flags & ECO_RT_KEEP_LOGITS) ? 1u : 0u;
  eco_world::TimedGraph t;
  t.n = n;
  HIPCHK(w, hipStreamBeginCapture(w->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  eco_status st = ECO_OK;
  for (uint32_t i = 0; i < n && st == ECO_OK; ++i) st = enqueue_step(w, w->cap_stream, d, w->ts, false);
  hipError_t e = hipStreamEndCapture(w->cap_stream, &t.graph);
  if (st != ECO_OK) {
    destroy_timed(t);
    return st;
  }
  const int u = (int)w->launch.unroll, H = (int)w->L.H1;
  const int mode = w->L.A + w->L.temp > 8 ? 2 : ((w->L.colour | w->L.ecology) != 0 ? 1 : 0);
  const void* fwd = w->L.wdtype == 0   ? forward_kernel_w0(H, u, mode)
                    : w->L.wdtype == 1 ? forward_kernel_w1(H, u, mode)
                                       : forward_kernel_w2(H, u, mode);
  size_t cnt = 0;
  if (e == hipSuccess) e = hipGraphGetNodes(t.graph, nullptr, &cnt);
  std::vector<hipGraphNode_t> nodes(cnt);
  if (e == hipSuccess && cnt) e = hipGraphGetNodes(t.graph, nodes.data(), &cnt);
  uint32_t found = 0;
  for (size_t i = 0; i < cnt && e == hipSuccess; ++i) {
    hipGraphNodeType ty;
    e = hipGraphNodeGetType(nodes[i], &ty);
    if (e != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams kp{};
    e = hipGraphKernelNodeGetParams(nodes[i], &kp);
    if (e != hipSuccess || kp.func != fwd) continue;
    const hipGraphNode_t f = nodes[i];
    size_t np = 0, nd = 0;
    e = hipGraphNodeGetDependencies(f, nullptr, &np);
    if (e == hipSuccess) e = hipGraphNodeGetDependentNodes(f, nullptr, &nd);
    std::vector<hipGraphNode_t> pre(np), post(nd);
    if (e == hipSuccess && np) e = hipGraphNodeGetDependencies(f, pre.data(), &np);
    if (e == hipSuccess && nd) e = hipGraphNodeGetDependentNodes(f, post.data(), &nd);
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) t.events.push_back(a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) t.events.push_back(b);
    hipGraphNode_t na = nullptr, nb = nullptr;
    // pre -> f  becomes  pre -> a -> f;  f -> post  becomes  f -> b -> post
    for (size_t j = 0; j < np && e == hipSuccess; ++j) e = hipGraphRemoveDependencies(t.graph, &pre[j], &f, 1);
    if (e == hipSuccess) e = hipGraphAddEventRecordNode(&na, t.graph, np ? pre.data() : nullptr, np, a);
    if (e == hipSuccess) e = hipGraphAddDependencies(t.graph, &na, &f, 1);
    for (size_t j = 0; j < nd && e == hipSuccess; ++j) e = hipGraphRemoveDependencies(t.graph, &f, &post[j], 1);
    if (e == hipSuccess) e = hipGraphAddEventRecordNode(&nb, t.graph, &f, 1, b);
    for (size_t j = 0; j < nd && e == hipSuccess; ++j) e = hipGraphAddDependencies(t.graph, &nb, &post[j], 1);
    if (e == hipSuccess) {
      t.pairs.push_back({ECO_K_FORWARD, {a, b}});
      ++found;
    }
  }
  if (e == hipSuccess && found != n) {
    destroy_timed(t);
    return fail(ECO_EDEVICE, "timed graph: policy-kernel nodes not found in the capture");
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&t.exec, t.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    destroy_timed(t);
    return dev_fail(w, e, "timed graph");
  }
  w->tgraphs.push_back(std::move(t));
  *out = &w->tgraphs.back();
  return ECO_OK;
}

eco_status check_world(const eco_world* w) {
  if (!w) return fail(ECO_EINVAL, "null world");
  if (w->broken) return fail(ECO_ESTATE, "world is in error state; call eco_world_reset");
  return ECO_OK;
}

// Host copy of the layout's unit mapping (read/write of weights in logical order).
struct HostUnit {
  uint32_t p, nvalid, row, kb;
  int layer;
};
HostUnit host_unit(const Layout& L, uint32_t u) {
  HostUnit r{};
  if (u < L.u_b1) { r.layer = 0; r.kb = u / L.H1; r.row = u % L.H1; r.p = L.p_w1 + r.row * L.D + 4 * r.kb; r.nvalid = 4; }
  else if (u < L.u_w2) { r.layer = 3; r.row = 4 * (u - L.u_b1); r.p = L.p_b1 + r.row; r.nvalid = 4; }
  else if (u < L.u_b2) { uint32_t e = u - L.u_w2; r.layer = 1; r.kb = e / L.H2; r.row = e % L.H2; r.p = L.p_w2 + r.row * L.H1 + 4 * r.kb; r.nvalid = 4; }
  else if (u < L.u_w3) { r.layer = 4; r.row = 4 * (u - L.u_b2); r.p = L.p_b2 + r.row; r.nvalid = 4; }
  else if (u < L.u_b3) { uint32_t e = u - L.u_w3, per = L.H2 / 4; r.layer = 2; r.row = e / per; r.kb = e % per; r.p = L.p_w3 + r.row * L.H2 + 4 * r.kb; r.nvalid = r.row < L.A ? 4 : 0; }
  else { uint32_t e = u - L.u_b3, n3 = L.A + L.temp; r.layer = 5; r.row = 4 * e; r.p = L.p_b3 + r.row; r.nvalid = r.row < n3 ? std::min(4u, n3 - r.row) : 0; }
  return r;
}

double host_fp8(uint8_t q) {
  const int e = (q >> 3) & 15, m = q & 7;
  double v = (e == 0) ? std::ldexp((double)m, -9) : std::ldexp(1.0 + m / 8.0, e - 7);
  return (q & 0x80) ? -v : v;
}

double host_bf16(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* eco_last_error(void) { return g_err.c_str(); }

eco_status eco_world_create(const eco_world_desc* descs, uint32_t n_worlds, void* hip_stream,
                            const eco_allocator* alloc, eco_world** out) {
  if (!out) return fail(ECO_EINVAL, "out is NULL");
  *out = nullptr;
  if (!descs || n_worlds == 0) return fail(ECO_EINVAL, "no worlds");
  if (n_worlds > kMaxWorldsH) return fail(ECO_EINVAL, "n_worlds exceeds 1024");
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(ECO_EINVAL, "allocator needs alloc and free");
  for (uint32_t i = 0; i < n_worlds; ++i) {
    eco_status st = check_desc(descs[i], i);
    if (st != ECO_OK) return st;
    const eco_world_desc& a = descs[0];
    const eco_world_desc& b = descs[i];
    if (a.window != b.window || a.n_scalars != b.n_scalars || a.hidden1 != b.hidden1 || a.hidden2 != b.hidden2 ||
        a.n_actions != b.n_actions || a.wdtype != b.wdtype || a.flags != b.flags)
      return fail(ECO_EINVAL, "all worlds of one object need the same window, n_scalars, hidden sizes, "
                              "n_actions, wdtype and flags");
  }
  eco_world* w = new eco_world();
  w->n_worlds = n_worlds;
  w->descs.assign(descs, descs + n_worlds);
  w->stream = (hipStream_t)hip_stream;
  if (alloc) {
    w->has_alloc = true;
    w->alloc = *alloc;
  }
  make_layout(descs[0], w->L, w->std1, w->std2, w->std3);
  int dev = 0;
  if (!alloc && hipGetDevice(&dev) != hipSuccess) {   // (with the caller's allocator: after allocating)
    (void)hipGetLastError();
    delete w;
    return fail(ECO_EDEVICE, "no HIP device");
  }
  // world tables: slot and cell ranges aligned to 64
  uint64_t so = 0, co = 0;
  w->wp.resize(n_worlds);
  bool any_attack = false;
  for (uint32_t i = 0; i < n_worlds; ++i) {
    const eco_world_desc& d = descs[i];
    WorldParams& p = w->wp[i];
    p = WorldParams{};
    p.W = d.width;
    p.H = d.height;
    p.cells = d.width * d.height;
    p.cap = d.capacity;
    p.slot_off = (uint32_t)so;
    p.cell_off = (uint32_t)co;
    p.regrow_thr = bern_threshold(d.regrow_prob);
    p.density_thr = bern_threshold(d.resource_density);
    p.e_init = d.e_init;
    p.e_cost = d.e_cost;
    p.e_eat = d.e_eat;
    p.e_repro = d.e_repro;
    p.e_child = d.e_child;
    p.sigma = d.mutation_sigma;
    p.n_init = d.n_agents_init;
    p.has_walls = 0;
    p.attack = d.attack_enabled;
    any_attack |= d.attack_enabled != 0;
    w->tile_rng_h.push_back(w->n_slot_tiles);
    for (uint32_t s = 0; s < p.cap; s += kSlotTileH) {
      w->slot_tiles_h.push_back(Tile{i, s, std::min(kSlotTileH, p.cap - s), 0});
      ++w->n_slot_tiles;
    }
    w->tile_rng_h.push_back(w->n_slot_tiles);
    w->tile_rng_h.push_back(w->n_cell_tiles);
    for (uint32_t c = 0; c < p.cells; c += kCellTileH) {
      w->cell_tiles_h.push_back(Tile{i, c, std::min(kCellTileH, p.cells - c), 0});
      ++w->n_cell_tiles;
    }
    w->tile_rng_h.push_back(w->n_cell_tiles);
    so = round_up(so + p.cap, 64);
    co = round_up(co + p.cells, 64);
  }
  if (so >= (1ull << 31) || co >= (1ull << 31)) {
    delete w;
    return fail(ECO_EINVAL, "total slots or cells exceed 2^31");
  }
  w->total_slots = (uint32_t)so;
  w->total_cells = (uint32_t)co;
  upload_world_params(w);

  // allocations
  Dev& d = w->d;
  const uint64_t TS = so, TC = co;
  bool ok = true;
  auto A = [&](size_t bytes) -> void* {
    void* p = ok ? dalloc(w, bytes) : nullptr;
    if (!p) ok = false;
    return p;
  };
  d.wp = (const WorldParams*)A(sizeof(WorldParams) * n_worlds);
  d.wv = (WorldVar*)A(sizeof(WorldVar) * n_worlds);
  d.cnt = (StepCounters*)A(sizeof(StepCounters) * n_worlds);
  d.ring = (eco_stats*)A(sizeof(eco_stats) * kStatsRing * n_worlds);
  d.pos = (int32_t*)A(4 * TS);
  d.energy = (int32_t*)A(4 * TS);
  d.age = (int32_t*)A(4 * TS);
  d.tgt = (int32_t*)A(4 * TS);
  d.facing = (uint8_t*)A(TS);
  d.flags = (uint8_t*)A(TS);
  d.act = (uint8_t*)A(TS);
  d.sampled = (uint8_t*)A(TS);
  d.act_in = (uint8_t*)A(TS);
  d.uid = (unsigned long long*)A(8 * TS);
  d.puid = (unsigned long long*)A(8 * TS);
  d.trait = (double*)A(8 * TS);
  d.occ = (int32_t*)A(4 * TC);
  d.claim = (uint32_t*)A(4 * TC);
  d.mark = any_attack ? (uint32_t*)A(4 * TC) : nullptr;
  d.res = (uint8_t*)A(TC);
  d.wall = (uint8_t*)A(TC);
  d.sense = (uint8_t*)A(TC);
  d.rgb = (w->L.colour || w->L.ecology) ? (uint32_t*)A(4 * TC) : nullptr;
  if (w->L.ecology) {
    d.ep = (const eco_ecology*)A(sizeof(eco_ecology) * n_worlds);
    d.water = (int32_t*)A(4 * TS);
    d.biomass = (int32_t*)A(4 * TS);
    d.hp = (int32_t*)A(4 * TS);
    d.cw = (int32_t*)A(4 * TC);
    d.ce = (int32_t*)A(4 * TC);
    d.cb = (int32_t*)A(4 * TC);
    if (descs[0].flags & ECO_DESC_TERRAIN) {
      d.rock = (int32_t*)A(4 * TC);
      d.flowdir = (int8_t*)A(TC);
      d.cw_next = (int32_t*)A(4 * TC);
    }
  }
  d.colour = w->L.colour ? (float4*)A(16 * TS) : nullptr;
  d.live = (int32_t*)A(4 * TS);
  d.bparent = (int32_t*)A(4 * TS);
  d.freel = (int32_t*)A(4 * TS);
  d.lgs = w->L.R3;
  d.logits = (float*)A(4ull * d.lgs * TS);
  d.trig = (const double2*)A(sizeof(double2) * kTrigTable);
  d.cellkeys = (unsigned long long*)A(8 * TC);
  d.sorted = (unsigned long long*)A(8 * TC);
  d.store = (uint8_t*)A(w->L.sstride * TS);
  d.master = (w->L.wdtype == ECO_W_FP32) ? d.store : (uint8_t*)A(w->L.mstride * TS);
  w->slot_tiles = (Tile*)A(sizeof(Tile) * std::max<size_t>(1, w->slot_tiles_h.size()));
  w->cell_tiles = (Tile*)A(sizeof(Tile) * std::max<size_t>(1, w->cell_tiles_h.size()));
  w->part_slot = (uint32_t*)A(4ull * kSlotPartH * std::max(1u, w->n_slot_tiles));
  w->part_cell = (unsigned long long*)A(8ull * kCellPartH * std::max(1u, w->n_cell_tiles));
  w->tile_rng = (uint32_t*)A(4ull * w->tile_rng_h.size());
  {
    const uint64_t T = std::max(1u, w->n_slot_tiles);
    TileScratch& ts = w->ts;
    ts.slot_tiles = w->slot_tiles;
    ts.cell_tiles = w->cell_tiles;
    ts.tile_rng = w->tile_rng;
    ts.n_slot_tiles = w->n_slot_tiles;
    ts.n_cell_tiles = w->n_cell_tiles;
    ts.part_slot = w->part_slot;
    ts.part_cell = w->part_cell;
    ts.scan = (uint32_t*)A(16 * T);
    ts.esum = (long long*)A(8 * T);
    ts.ecosum = w->L.ecology ? (unsigned long long*)A(3 * 8 * T) : nullptr;
    ts.tmean = (double*)A(8 * T);
    ts.tm2 = (double*)A(8 * T);
  }
  w->emit_list = (uint32_t*)A(8 * TS);
  {   // placement buckets: 2^k per world, about four cells each
    std::vector<uint32_t> pinfo;
    uint32_t nb = 0;
    for (uint32_t i = 0; i < n_worlds; ++i) {
      uint32_t k = 0;
      while (k < 30 && (4ull << k) < w->wp[i].cells) ++k;
      pinfo.push_back(nb);
      pinfo.push_back(32 - k);
      nb += 1u << k;
    }
    pinfo.push_back(nb);
    pinfo.push_back(32);
    w->n_buckets = nb;
    w->place_info = A(4 * pinfo.size());
    w->place_cnt = (uint32_t*)A(4ull * nb);
    w->place_start = (uint32_t*)A(4ull * (nb + n_worlds));
    w->place_info_h = pinfo;
  }
  if (!ok) {
    free_all(w);
    delete w;
    return fail(ECO_ENOMEM, "device allocation failed");
  }
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&w->n_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      birth_commit_blocks_per_cu(w->L, &w->birth_bpc) != hipSuccess) {
    (void)hipGetLastError();
    free_all(w);
    delete w;
    return fail(ECO_EDEVICE, "no HIP device");
  }
  w->birth_bpc = std::max(1, w->birth_bpc);
  d.n_worlds = n_worlds;
  d.total_slots = w->total_slots;
  d.total_cells = w->total_cells;
  d.keep_logits = 0;
  d.inject = 0;
  d.dry = 0;
  hipStream_t s = w->stream;
  eco_status st = ECO_OK;
  auto chk = [&](hipError_t e, const char* what) {
    if (st == ECO_OK && e != hipSuccess) st = dev_fail(w, e, what);
  };
  chk(hipStreamCreateWithFlags(&w->cap_stream, hipStreamNonBlocking), "create capture stream");
  chk(hipMemcpyAsync(w->slot_tiles, w->slot_tiles_h.data(), sizeof(Tile) * w->slot_tiles_h.size(),
                     hipMemcpyHostToDevice, s), "upload tiles");
  chk(hipMemcpyAsync(w->cell_tiles, w->cell_tiles_h.data(), sizeof(Tile) * w->cell_tiles_h.size(),
                     hipMemcpyHostToDevice, s), "upload tiles");
  chk(hipMemcpyAsync(w->tile_rng, w->tile_rng_h.data(), 4 * w->tile_rng_h.size(), hipMemcpyHostToDevice, s),
      "upload tile ranges");
  chk(hipMemcpyAsync(w->place_info, w->place_info_h.data(), 4 * w->place_info_h.size(), hipMemcpyHostToDevice, s),
      "upload placement table");
  {
    static const std::vector<double2> trig = angle_table();
    chk(hipMemcpyAsync((void*)d.trig, trig.data(), sizeof(double2) * kTrigTable, hipMemcpyHostToDevice, s),
        "upload angle table");
  }
  chk(hipMemsetAsync(d.store, 0, w->L.sstride * TS, s), "clear weights");
  if (d.master != d.store) chk(hipMemsetAsync(d.master, 0, w->L.mstride * TS, s), "clear master");
  chk(hipMemsetAsync(d.trait, 0, 8 * TS, s), "clear trait");
  chk(hipMemsetAsync(d.sampled, 0xFF, TS, s), "clear sampled");
  chk(hipMemsetAsync(d.act_in, 0, TS, s), "clear act_in");
  chk(hipMemsetAsync(w->part_slot, 0, 4ull * kSlotPartH * std::max(1u, w->n_slot_tiles), s), "clear partials");
  chk(hipMemsetAsync(w->part_cell, 0, 8ull * kCellPartH * std::max(1u, w->n_cell_tiles), s), "clear partials");
  chk(hipMemsetAsync(d.cnt, 0, sizeof(StepCounters) * n_worlds, s), "clear counters");
  if (d.ep) {
    std::vector<eco_ecology> ep(n_worlds);
    for (uint32_t i = 0; i < n_worlds; ++i) ep[i] = descs[i].eco;
    chk(hipMemcpyAsync((void*)d.ep, ep.data(), sizeof(eco_ecology) * n_worlds, hipMemcpyHostToDevice, s),
        "upload ecology parameters");
    chk(hipStreamSynchronize(s), "upload ecology parameters");
  }
  if (st == ECO_OK) st = run_init(w);
  if (st != ECO_OK) {
    std::string msg = g_err;
    eco_world_destroy(w);
    g_err = msg;
    return st;
  }
  *out = w;
  return ECO_OK;
}

void eco_world_destroy(eco_world* w) {
  if (!w) return;
  (void)hipStreamSynchronize(w->stream);
  drop_graph(w);
  for (auto e : w->ev_pool) (void)hipEventDestroy(e);
  if (w->cap_stream) (void)hipStreamDestroy(w->cap_stream);
  free_all(w);
  delete w;
}

eco_status eco_world_step(eco_world* w, uint32_t n_steps) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (n_steps == 0) return ECO_OK;
  const bool timed = (w->rt_flags & ECO_RT_TIME_KERNELS) != 0;
  const bool graph = (w->rt_flags & ECO_RT_USE_GRAPH) != 0;
  Dev d = w->d;
  d.inject = 0;
  d.dry = 0;
  d.keep_logits = (w->rt_flags & ECO_RT_KEEP_LOGITS) ? 1u : 0u;
  if (graph && timed) {
    eco_world::TimedGraph* t = nullptr;
    st = timed_graph(w, n_steps, &t);
    if (st != ECO_OK) return st;
    HIPCHK(w, hipGraphLaunch(t->exec, w->stream), "graph launch");
    w->ev_pending.insert(w->ev_pending.end(), t->pairs.begin(), t->pairs.end());
    return drain_events(w);
  }
  if (graph) {
    for (uint32_t left = n_steps; left > 0;) {
      const uint32_t m = std::min(left, kGraphSteps);
      hipGraphExec_t ex = nullptr;
      st = step_graph(w, m, &ex);
      if (st != ECO_OK) return st;
      HIPCHK(w, hipGraphLaunch(ex, w->stream), "graph launch");
      left -= m;
    }
    return ECO_OK;
  }
  for (uint32_t i = 0; i < n_steps; ++i) {
    st = enqueue_step(w, w->stream, d, w->ts, timed);
    if (st != ECO_OK) return st;
  }
  if (timed) return drain_events(w);
  return ECO_OK;
}

eco_status eco_world_step_static(eco_world* w, uint32_t n_steps) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (n_steps == 0) return ECO_OK;
  // the step's scratch, laid out in the static array (each part 256-aligned)
  const uint64_t T = std::max(1u, w->n_slot_tiles), C = std::max(1u, w->n_cell_tiles);
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off = round_up(off + bytes, 256);
    return o;
  };
  const uint64_t o_part_slot = take(4ull * kSlotPartH * T), o_part_cell = take(8ull * kCellPartH * C),
                 o_scan = take(16 * T), o_esum = take(8 * T), o_tmean = take(8 * T), o_tm2 = take(8 * T),
                 o_ecosum = w->L.ecology ? take(24 * T) : 0, o_bparent = take(4ull * w->total_slots),
                 o_freel = take(4ull * w->total_slots), o_cnt = take(sizeof(StepCounters) * w->n_worlds);
  void* base = nullptr;
  size_t cap = 0;
  HIPCHK(w, static_scratch(&base, &cap), "static scratch address");
  if (off > cap) {
    char buf[200];
    snprintf(buf, sizeof buf, "eco_world_step_static: the object needs %llu bytes of scratch, above the static "
             "array's %llu", (unsigned long long)off, (unsigned long long)cap);
    return fail(ECO_EINVAL, buf);
  }
  uint8_t* b = static_cast<uint8_t*>(base);
  Dev d = w->d;
  d.inject = 0;
  d.dry = 0;
  d.keep_logits = (w->rt_flags & ECO_RT_KEEP_LOGITS) ? 1u : 0u;
  d.bparent = reinterpret_cast<int32_t*>(b + o_bparent);
  d.freel = reinterpret_cast<int32_t*>(b + o_freel);
  d.cnt = reinterpret_cast<StepCounters*>(b + o_cnt);
  TileScratch ts = w->ts;
  ts.part_slot = reinterpret_cast<uint32_t*>(b + o_part_slot);
  ts.part_cell = reinterpret_cast<unsigned long long*>(b + o_part_cell);
  ts.scan = reinterpret_cast<uint32_t*>(b + o_scan);
  ts.esum = reinterpret_cast<long long*>(b + o_esum);
  ts.tmean = reinterpret_cast<double*>(b + o_tmean);
  ts.tm2 = reinterpret_cast<double*>(b + o_tm2);
  ts.ecosum = w->L.ecology ? reinterpret_cast<unsigned long long*>(b + o_ecosum) : nullptr;
  // every part is written by the step before it is read (the tile counters by
  // the move, claim and compaction passes, the birth lists and counters by the
  // ranking pass), so nothing needs clearing between calls
  for (uint32_t i = 0; i < n_steps; ++i) {
    st = enqueue_step(w, w->stream, d, ts, false);
    if (st != ECO_OK) return st;
  }
  return ECO_OK;
}

eco_status eco_world_prepare(eco_world* w, uint32_t n_steps) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (!(w->rt_flags & ECO_RT_USE_GRAPH)) return ECO_OK;
  if (w->rt_flags & ECO_RT_TIME_KERNELS) {
    if (n_steps == 0) return ECO_OK;
    eco_world::TimedGraph* t = nullptr;
    return timed_graph(w, n_steps, &t);
  }
  return prepare_step_graphs(w, n_steps);
}

eco_status eco_world_step_with_actions(eco_world* w, const uint8_t* actions) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (!actions) return fail(ECO_EINVAL, "actions is NULL");
  // validate against the live slots
  std::vector<uint8_t> flags(w->total_slots), act(w->total_slots, 0);
  HIPCHK(w, hipMemcpyAsync(flags.data(), w->d.flags, w->total_slots, hipMemcpyDeviceToHost, w->stream), "read flags");
  st = sync(w);
  if (st != ECO_OK) return st;
  uint64_t k = 0;
  for (uint32_t i = 0; i < w->n_worlds; ++i) {
    const WorldParams& p = w->wp[i];
    for (uint32_t s = 0; s < p.cap; ++s, ++k) {
      const uint8_t a = actions[k];
      if ((flags[p.slot_off + s] & kAlive) && a >= w->L.A) return fail(ECO_EINVAL, "action out of range for a live slot");
      act[p.slot_off + s] = a;
    }
  }
  HIPCHK(w, hipMemcpyAsync(w->d.act_in, act.data(), w->total_slots, hipMemcpyHostToDevice, w->stream), "upload actions");
  Dev d = w->d;
  d.inject = 1;
  d.dry = 0;
  d.keep_logits = (w->rt_flags & ECO_RT_KEEP_LOGITS) ? 1u : 0u;
  st = enqueue_step(w, w->stream, d, w->ts, false);
  if (st != ECO_OK) return st;
  return sync(w);
}

eco_status eco_world_reset(eco_world* w, const uint64_t* seeds) {
  if (!w) return fail(ECO_EINVAL, "null world");
  (void)hipGetLastError();
  if (seeds)
    for (uint32_t i = 0; i < w->n_worlds; ++i) w->descs[i].seed = seeds[i];
  upload_world_params(w);
  hipStream_t s = w->stream;
  Dev& d = w->d;
  w->broken = false;
  HIPCHK(w, hipMemsetAsync(d.store, 0, w->L.sstride * (uint64_t)w->total_slots, s), "clear weights");
  if (d.master != d.store) HIPCHK(w, hipMemsetAsync(d.master, 0, w->L.mstride * (uint64_t)w->total_slots, s), "clear master");
  HIPCHK(w, hipMemsetAsync(d.trait, 0, 8ull * w->total_slots, s), "clear trait");
  return run_init(w);
}

eco_status eco_world_stats(eco_world* w, eco_stats* out, uint32_t max_worlds) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (!out) return fail(ECO_EINVAL, "out is NULL");
  const uint32_t n = std::min(max_worlds, w->n_worlds);
  std::vector<WorldVar> wv(w->n_worlds);
  HIPCHK(w, hipMemcpyAsync(wv.data(), w->d.wv, sizeof(WorldVar) * w->n_worlds, hipMemcpyDeviceToHost, w->stream), "read vars");
  st = sync(w);
  if (st != ECO_OK) return st;
  for (uint32_t i = 0; i < n; ++i)
    HIPCHK(w, hipMemcpyAsync(out + i, w->d.ring + (uint64_t)i * kStatsRing + wv[i].step % kStatsRing, sizeof(eco_stats),
                             hipMemcpyDeviceToHost, w->stream), "read stats");
  return sync(w);
}

eco_status eco_world_stats_history(eco_world* w, uint32_t world, eco_stats* out, uint32_t max_records, uint32_t* n_out) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (!out || !n_out || world >= w->n_worlds) return fail(ECO_EINVAL, "bad arguments");
  WorldVar v;
  HIPCHK(w, hipMemcpyAsync(&v, w->d.wv + world, sizeof v, hipMemcpyDeviceToHost, w->stream), "read vars");
  st = sync(w);
  if (st != ECO_OK) return st;
  const uint64_t avail = std::min<uint64_t>(v.step + 1, kStatsRing);
  const uint32_t n = (uint32_t)std::min<uint64_t>(avail, max_records);
  std::vector<eco_stats> ring(kStatsRing);
  HIPCHK(w, hipMemcpyAsync(ring.data(), w->d.ring + (uint64_t)world * kStatsRing, sizeof(eco_stats) * kStatsRing,
                           hipMemcpyDeviceToHost, w->stream), "read ring");
  st = sync(w);
  if (st != ECO_OK) return st;
  for (uint32_t i = 0; i < n; ++i) out[i] = ring[(v.step - (n - 1) + i) % kStatsRing];
  *n_out = n;
  return ECO_OK;
}

eco_status eco_world_info(const eco_world* w, eco_info* out) {
  if (!w || !out) return fail(ECO_EINVAL, "null argument");
  eco_info i{};
  i.n_worlds = w->n_worlds;
  i.total_slots = w->total_slots;
  i.total_cells = w->total_cells;
  i.input_dim = w->L.D;
  i.hidden1 = w->L.H1;
  i.hidden2 = w->L.H2;
  i.n_actions = w->L.A;
  i.param_count = w->L.P;
  i.weight_bytes_per_agent = weight_bytes(w->L);
  i.storage_stride = w->L.sstride;
  i.master_stride = (w->L.wdtype == ECO_W_FP32) ? 0 : w->L.mstride;
  i.device_bytes = w->device_bytes;
  i.n_cus = (uint32_t)w->n_cus;
  i.wdtype = w->L.wdtype;
  *out = i;
  return ECO_OK;
}

eco_status eco_world_set_flags(eco_world* w, uint32_t flags) {
  if (!w) return fail(ECO_EINVAL, "null world");
  if (flags & ~(ECO_RT_KEEP_LOGITS | ECO_RT_USE_GRAPH | ECO_RT_TIME_KERNELS | ECO_RT_SPLIT_STEP))
    return fail(ECO_EINVAL, "unknown flag");
  if (flags != w->rt_flags) drop_graph(w);
  w->rt_flags = flags;
  return ECO_OK;
}

eco_status eco_world_set_launch(eco_world* w, const eco_launch* lc) {
  if (!w || !lc) return fail(ECO_EINVAL, "null argument");
  const uint32_t wpb = lc->waves_per_block, u = lc->unroll;
  if (!(wpb == 1 || wpb == 2 || wpb == 4 || wpb == 8)) return fail(ECO_EINVAL, "waves_per_block must be 1, 2, 4 or 8");
  if (!(u == 4 || u == 8 || u == 16)) return fail(ECO_EINVAL, "unroll must be 4, 8 or 16");
  if (lc->blocks_per_cu < 1 || lc->blocks_per_cu > 64) return fail(ECO_EINVAL, "blocks_per_cu must be in 1..64");
  if (forward_shmem(w, wpb) > 64 * 1024) return fail(ECO_EINVAL, "launch needs more than 64 KiB of LDS per block");
  w->launch = *lc;
  w->launch.reserved = 0;
  drop_graph(w);
  return ECO_OK;
}

eco_status eco_world_get_launch(const eco_world* w, eco_launch* out) {
  if (!w || !out) return fail(ECO_EINVAL, "null argument");
  *out = w->launch;
  return ECO_OK;
}

eco_status eco_world_autotune(eco_world* w, eco_launch* best) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  Dev d = w->d;
  d.dry = 1;
  d.inject = 0;
  d.keep_logits = 0;
  std::vector<eco_launch> cand;
  const uint32_t wpbs[] = {1, 2, 4, 8}, us[] = {4, 8, 16}, bpcs[] = {1, 2, 4, 8, 16};
  for (uint32_t wpb : wpbs)
    for (uint32_t u : us)
      for (uint32_t bpc : bpcs) {
        if (wpb * bpc > 32 || wpb * bpc < 4) continue;  // 4..32 waves per CU
        if (forward_shmem(w, wpb) > 64 * 1024 || forward_shmem(w, wpb) * bpc > 160 * 1024) continue;
        cand.push_back(eco_launch{wpb, bpc, u, 0});
      }
  // Rounds over the candidates, each timed over `reps` consecutive launches per
  // round: drifts of clock or memory state during tuning hit every shape alike.
  // The first pass (one launch, median over rounds) keeps the four fastest; the
  // second times those as runs of three launches, as a step loop repeats one
  // shape, and ranks them by the mean over more rounds, the statistic a step's
  // cost follows (a median hides a shape that is only sometimes slow).
  auto timings = [&](const std::vector<eco_launch>& c, int rounds, int reps, bool mean,
                     std::vector<float>& score) -> hipError_t {
    const size_t n = c.size();
    std::vector<hipEvent_t> ev(n + 1, nullptr);
    hipError_t e = hipSuccess;
    for (auto& x : ev)
      if (e == hipSuccess) e = hipEventCreate(&x);
    for (size_t i = 0; i < n && e == hipSuccess; ++i) e = launch_forward(w, w->stream, d, c[i]);  // warm-up
    std::vector<std::vector<float>> t(n);
    for (int r = 0; r < rounds && e == hipSuccess; ++r) {
      e = hipEventRecord(ev[0], w->stream);
      for (size_t i = 0; i < n && e == hipSuccess; ++i) {
        for (int k = 0; k < reps && e == hipSuccess; ++k) e = launch_forward(w, w->stream, d, c[i]);
        if (e == hipSuccess) e = hipEventRecord(ev[i + 1], w->stream);
      }
      if (e == hipSuccess) e = hipEventSynchronize(ev[n]);
      for (size_t i = 0; i < n && e == hipSuccess; ++i) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        t[i].push_back(ms / (float)reps);
      }
    }
    for (auto& x : ev)
      if (x) (void)hipEventDestroy(x);
    score.assign(n, 1e30f);
    for (size_t i = 0; i < n && e == hipSuccess; ++i) {
      std::sort(t[i].begin(), t[i].end());
      double sum = 0.0;
      for (float v : t[i]) sum += v;
      score[i] = mean ? (float)(sum / (double)t[i].size()) : t[i][t[i].size() / 2];
    }
    return e;
  };
  std::vector<float> med1, med2;
  hipError_t e = timings(cand, 9, 1, false, med1);
  if (e != hipSuccess) return dev_fail(w, e, "autotune");
  std::vector<size_t> order(cand.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return med1[a] < med1[b]; });
  std::vector<eco_launch> top;
  for (size_t i = 0; i < order.size() && i < 4; ++i) top.push_back(cand[order[i]]);
  e = timings(top, 11, 3, true, med2);
  if (e != hipSuccess) return dev_fail(w, e, "autotune");
  eco_launch chosen = w->launch;
  float best_ms = 1e30f;
  for (size_t i = 0; i < top.size(); ++i) {
    if (med2[i] < best_ms) {
      best_ms = med2[i];
      chosen = top[i];
    }
  }
  w->launch = chosen;
  drop_graph(w);
  if (best) *best = chosen;
  return ECO_OK;
}

eco_status eco_world_autotune_cached(eco_world* w, const char* path, eco_launch* best, int* from_cache) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (!path) return fail(ECO_EINVAL, "autotune cache path is NULL");
  // the key: device, policy shape, live population (power-of-two bucket)
  int dev = 0;
  hipDeviceProp_t prop;
  HIPCHK(w, hipGetDevice(&dev), "hipGetDevice");
  HIPCHK(w, hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
  std::string arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  std::vector<WorldVar> wv(w->n_worlds);
  HIPCHK(w, hipMemcpyAsync(wv.data(), w->d.wv, sizeof(WorldVar) * w->n_worlds, hipMemcpyDeviceToHost, w->stream),
         "read vars");
  st = sync(w);
  if (st != ECO_OK) return st;
  uint64_t live = 0;
  for (const auto& v : wv) live += v.n_live;
  uint32_t lg = 0;
  while ((2ull << lg) <= live) ++lg;   // live in [2^lg, 2^(lg+1)), 0 for none or one
  const int words = (w->L.colour | w->L.ecology) != 0, nine = w->L.A + w->L.temp > 8;
  char key[200];
  snprintf(key, sizeof key, "%s cus=%d D=%u H=%u A=%u S=%u wdtype=%u words=%d nine=%d live=2^%u", arch.c_str(),
           w->n_cus, w->L.D, w->L.H1, w->L.A, w->L.S, w->L.wdtype, words, nine, lg);
  if (FILE* f = std::fopen(path, "r")) {
    char line[512];
    eco_launch hit{};
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
      char k[200];
      unsigned a = 0, b = 0, c = 0;
      if (std::sscanf(line, " {\"key\": \"%199[^\"]\", \"waves_per_block\": %u, \"blocks_per_cu\": %u, \"unroll\": %u",
                      k, &a, &b, &c) == 4 &&
          std::strcmp(k, key) == 0) {
        hit = eco_launch{a, b, c, 0};
        found = true;   // the last matching line wins
      }
    }
    std::fclose(f);
    if (found) {
      st = eco_world_set_launch(w, &hit);
      if (st != ECO_OK) return st;
      if (best) *best = hit;
      if (from_cache) *from_cache = 1;
      return ECO_OK;
    }
  }
  eco_launch chosen{};
  st = eco_world_autotune(w, &chosen);
  if (st != ECO_OK) return st;
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "{\"key\": \"%s\", \"waves_per_block\": %u, \"blocks_per_cu\": %u, \"unroll\": %u}\n", key,
                 chosen.waves_per_block, chosen.blocks_per_cu, chosen.unroll);
    std::fclose(f);
  }
  if (best) *best = chosen;
  if (from_cache) *from_cache = 0;
  return ECO_OK;
}

eco_status eco_world_kernel_times(eco_world* w, eco_kernel_times* out, int reset) {
  if (!w) return fail(ECO_EINVAL, "null world");
  eco_status st = drain_events(w);
  if (st != ECO_OK) return st;
  if (out) *out = w->kt;
  if (reset) w->kt = eco_kernel_times{};
  return ECO_OK;
}

size_t eco_world_state_bytes(const eco_world* w, uint32_t world) {
  if (!w || world >= w->n_worlds) return 0;
  const uint64_t cap = w->wp[world].cap, cells = w->wp[world].cells;
  return 32 + cap * (8 + 8 + 4 + 4 + 4 + 1 + 1 + 1) + cells * (4 + 1 + 1) + (w->L.ecology ? 12 * (cap + cells) : 0);
}

eco_status eco_world_read_state(eco_world* w, uint32_t world, void* buf, size_t bytes) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (world >= w->n_worlds || !buf) return fail(ECO_EINVAL, "bad world or buffer");
  if (bytes < eco_world_state_bytes(w, world)) return fail(ECO_EINVAL, "state buffer too small");
  const WorldParams& p = w->wp[world];
  const size_t cap = p.cap, cells = p.cells;
  uint8_t* b = (uint8_t*)buf;
  WorldVar v;
  std::vector<uint8_t> flags(cap);
  hipStream_t s = w->stream;
  HIPCHK(w, hipMemcpyAsync(&v, w->d.wv + world, sizeof v, hipMemcpyDeviceToHost, s), "read vars");
  uint8_t* q = b + 32;
  auto cp = [&](const void* src, size_t n) -> hipError_t {
    hipError_t e = hipMemcpyAsync(q, src, n, hipMemcpyDeviceToHost, s);
    q += n;
    return e;
  };
  HIPCHK(w, cp(w->d.uid + p.slot_off, cap * 8), "read uid");
  HIPCHK(w, cp(w->d.puid + p.slot_off, cap * 8), "read puid");
  HIPCHK(w, cp(w->d.pos + p.slot_off, cap * 4), "read pos");
  HIPCHK(w, cp(w->d.energy + p.slot_off, cap * 4), "read energy");
  HIPCHK(w, cp(w->d.age + p.slot_off, cap * 4), "read age");
  HIPCHK(w, cp(w->d.occ + p.cell_off, cells * 4), "read occ");
  HIPCHK(w, cp(w->d.facing + p.slot_off, cap), "read facing");
  uint8_t* alive = q;
  HIPCHK(w, cp(w->d.flags + p.slot_off, cap), "read flags");
  HIPCHK(w, cp(w->d.act + p.slot_off, cap), "read action");
  HIPCHK(w, cp(w->d.res + p.cell_off, cells), "read res");
  HIPCHK(w, cp(w->d.wall + p.cell_off, cells), "read wall");
  if (w->L.ecology) {
    HIPCHK(w, cp(w->d.water + p.slot_off, cap * 4), "read water");
    HIPCHK(w, cp(w->d.biomass + p.slot_off, cap * 4), "read biomass");
    HIPCHK(w, cp(w->d.hp + p.slot_off, cap * 4), "read hp");
    HIPCHK(w, cp(w->d.cw + p.cell_off, cells * 4), "read cell water");
    HIPCHK(w, cp(w->d.ce + p.cell_off, cells * 4), "read cell energy");
    HIPCHK(w, cp(w->d.cb + p.cell_off, cells * 4), "read cell biomass");
  }
  st = sync(w);
  if (st != ECO_OK) return st;
  for (size_t i = 0; i < cap; ++i) alive[i] &= kAlive;
  const uint32_t hdr[4] = {p.W, p.H, p.cap, 0};
  std::memcpy(b, &v.step, 8);
  std::memcpy(b + 8, &v.uid_next, 8);
  std::memcpy(b + 16, hdr, 16);
  return ECO_OK;
}

eco_status eco_world_write_state(eco_world* w, uint32_t world, const void* buf, size_t bytes) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (world >= w->n_worlds || !buf) return fail(ECO_EINVAL, "bad world or buffer");
  if (bytes < eco_world_state_bytes(w, world)) return fail(ECO_EINVAL, "state buffer too small");
  const WorldParams& p = w->wp[world];
  const size_t cap = p.cap, cells = p.cells;
  const uint8_t* b = (const uint8_t*)buf;
  uint32_t hdr[4];
  std::memcpy(hdr, b + 16, 16);
  if (hdr[0] != p.W || hdr[1] != p.H || hdr[2] != p.cap) return fail(ECO_EINVAL, "state shape mismatch");
  // consistency: occ and pos describe the same placement
  const uint8_t* q = b + 32;
  const int32_t* pos = (const int32_t*)(q + cap * 16);
  const int32_t* occ = (const int32_t*)(q + cap * 28);
  const uint8_t* alive_new = q + cap * 28 + cells * 4 + cap;
  const uint8_t* facing = q + cap * 28 + cells * 4;
  for (size_t s = 0; s < cap; ++s) {
    if (alive_new[s] > 1) return fail(ECO_EINVAL, "alive must be 0 or 1");
    if (!alive_new[s]) continue;
    if (pos[s] < 0 || (uint32_t)pos[s] >= p.cells || occ[pos[s]] != (int32_t)s) return fail(ECO_EINVAL, "occ/pos mismatch");
    if (facing[s] > 3) return fail(ECO_EINVAL, "facing must be 0..3");
  }
  for (size_t c = 0; c < cells; ++c) {
    const int32_t o = occ[c];
    if (o < -1 || o >= (int32_t)cap || (o >= 0 && (!alive_new[o] || pos[o] != (int32_t)c)))
      return fail(ECO_EINVAL, "occ/pos mismatch");
  }
  const uint8_t* res = q + cap * 28 + cells * 4 + 3 * cap;
  const uint8_t* wall = res + cells;
  bool walls = false;
  for (size_t c = 0; c < cells; ++c) {
    if (res[c] > 1 || wall[c] > 1) return fail(ECO_EINVAL, "res and wall must be 0 or 1");
    walls |= wall[c] != 0;
  }
  if (w->L.ecology) {   // water, biomass, health per slot, then the grid's three layers
    const uint8_t* e8 = wall + cells;
    for (size_t i = 0; i < 3 * cap + 3 * cells; ++i) {
      int32_t v;
      std::memcpy(&v, e8 + 4 * i, 4);
      if (v < 0) return fail(ECO_EINVAL, "ecology amounts and health must be >= 0");
    }
  }
  std::vector<uint8_t> old(cap);
  hipStream_t s = w->stream;
  HIPCHK(w, hipMemcpyAsync(old.data(), w->d.flags + p.slot_off, cap, hipMemcpyDeviceToHost, s), "read flags");
  st = sync(w);
  if (st != ECO_OK) return st;
  WorldVar v;
  HIPCHK(w, hipMemcpyAsync(&v, w->d.wv + world, sizeof v, hipMemcpyDeviceToHost, s), "read vars");
  st = sync(w);
  if (st != ECO_OK) return st;
  std::memcpy(&v.step, b, 8);
  std::memcpy(&v.uid_next, b + 8, 8);
  v.n_births = 0;
  HIPCHK(w, hipMemcpyAsync(w->d.wv + world, &v, sizeof v, hipMemcpyHostToDevice, s), "write vars");
  auto cp = [&](void* dst, size_t n) -> hipError_t {
    hipError_t e = hipMemcpyAsync(dst, q, n, hipMemcpyHostToDevice, s);
    q += n;
    return e;
  };
  HIPCHK(w, cp(w->d.uid + p.slot_off, cap * 8), "write uid");
  HIPCHK(w, cp(w->d.puid + p.slot_off, cap * 8), "write puid");
  HIPCHK(w, cp(w->d.pos + p.slot_off, cap * 4), "write pos");
  HIPCHK(w, cp(w->d.energy + p.slot_off, cap * 4), "write energy");
  HIPCHK(w, cp(w->d.age + p.slot_off, cap * 4), "write age");
  HIPCHK(w, cp(w->d.occ + p.cell_off, cells * 4), "write occ");
  HIPCHK(w, cp(w->d.facing + p.slot_off, cap), "write facing");
  HIPCHK(w, cp(w->d.flags + p.slot_off, cap), "write alive");
  HIPCHK(w, cp(w->d.act + p.slot_off, cap), "write action");
  HIPCHK(w, cp(w->d.res + p.cell_off, cells), "write res");
  HIPCHK(w, cp(w->d.wall + p.cell_off, cells), "write wall");
  if (w->L.ecology) {
    HIPCHK(w, cp(w->d.water + p.slot_off, cap * 4), "write water");
    HIPCHK(w, cp(w->d.biomass + p.slot_off, cap * 4), "write biomass");
    HIPCHK(w, cp(w->d.hp + p.slot_off, cap * 4), "write hp");
    HIPCHK(w, cp(w->d.cw + p.cell_off, cells * 4), "write cell water");
    HIPCHK(w, cp(w->d.ce + p.cell_off, cells * 4), "write cell energy");
    HIPCHK(w, cp(w->d.cb + p.cell_off, cells * 4), "write cell biomass");
  }
  if (p.attack) HIPCHK(w, hipMemsetAsync(w->d.mark + p.cell_off, 0, cells * 4, s), "clear attack stamps");
  if (walls != (w->wp[world].has_walls != 0)) {
    w->wp[world].has_walls = walls ? 1u : 0u;
    HIPCHK(w, hipMemcpyAsync((void*)(w->d.wp + world), &w->wp[world], sizeof(WorldParams), hipMemcpyHostToDevice, s),
           "write world params");
  }
  std::vector<uint32_t> list;
  for (uint32_t sl = 0; sl < p.cap; ++sl)
    if (alive_new[sl] && !(old[sl] & kAlive)) {
      list.push_back(world);
      list.push_back(sl);
    }
  if (!list.empty()) {
    HIPCHK(w, hipMemcpyAsync(w->emit_list, list.data(), list.size() * 4, hipMemcpyHostToDevice, s), "upload list");
    HIPCHK(w, launch_emit_list(s, w->d, w->L, w->emit_list, (uint32_t)(list.size() / 2), EMIT_INIT, w->std1, w->std2,
                               w->std3, emit_blocks(w)), "init weights");
  }
  HIPCHK(w, launch_compact(s, w->d, w->ts, 1, (int)world), "compact");
  HIPCHK(w, launch_resource_total(s, w->d, (int)world), "resource total");
  return sync(w);
}

eco_status eco_world_read_logits(eco_world* w, uint32_t world, float* out, size_t n_floats) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (world >= w->n_worlds || !out) return fail(ECO_EINVAL, "bad world or buffer");
  const WorldParams& p = w->wp[world];
  if (n_floats < (size_t)p.cap * w->L.A) return fail(ECO_EINVAL, "logits buffer too small");
  const uint32_t lgs = w->d.lgs;
  std::vector<float> tmp((size_t)p.cap * lgs);
  HIPCHK(w, hipMemcpyAsync(tmp.data(), w->d.logits + (uint64_t)p.slot_off * lgs, tmp.size() * 4,
                           hipMemcpyDeviceToHost, w->stream), "read logits");
  st = sync(w);
  if (st != ECO_OK) return st;
  for (size_t s = 0; s < p.cap; ++s)
    for (uint32_t a = 0; a < w->L.A; ++a) out[s * w->L.A + a] = tmp[s * lgs + a];
  return ECO_OK;
}

eco_status eco_world_read_sampled(eco_world* w, uint32_t world, uint8_t* out, size_t n) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (world >= w->n_worlds || !out) return fail(ECO_EINVAL, "bad world or buffer");
  const WorldParams& p = w->wp[world];
  if (n < p.cap) return fail(ECO_EINVAL, "buffer too small");
  HIPCHK(w, hipMemcpyAsync(out, w->d.sampled + p.slot_off, p.cap, hipMemcpyDeviceToHost, w->stream), "read sampled");
  return sync(w);
}

eco_status eco_world_read_terrain(eco_world* w, uint32_t world, int32_t* rock, size_t n) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (world >= w->n_worlds || !rock) return fail(ECO_EINVAL, "bad world or buffer");
  if (!w->d.rock) return fail(ECO_EINVAL, "the object has no terrain (ECO_DESC_TERRAIN)");
  const WorldParams& p = w->wp[world];
  if (n < p.cells) return fail(ECO_EINVAL, "rock buffer too small");
  HIPCHK(w, hipMemcpyAsync(rock, w->d.rock + p.cell_off, 4ull * p.cells, hipMemcpyDeviceToHost, w->stream), "read rock");
  return sync(w);
}

eco_status eco_world_write_terrain(eco_world* w, uint32_t world, const int32_t* rock, size_t n) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (world >= w->n_worlds || !rock) return fail(ECO_EINVAL, "bad world or buffer");
  if (!w->d.rock) return fail(ECO_EINVAL, "the object has no terrain (ECO_DESC_TERRAIN)");
  const WorldParams& p = w->wp[world];
  if (n < p.cells) return fail(ECO_EINVAL, "rock buffer too small");
  for (size_t c = 0; c < p.cells; ++c)
    if (rock[c] < 0 || rock[c] > 31) return fail(ECO_EINVAL, "rock heights must lie in 0..31");
  hipStream_t s = w->stream;
  HIPCHK(w, hipMemcpyAsync(w->d.rock + p.cell_off, rock, 4ull * p.cells, hipMemcpyHostToDevice, s), "write rock");
  HIPCHK(w, launch_flowdir(s, w->d, w->ts, (int)world), "flow directions");
  HIPCHK(w, launch_render(s, w->d, w->ts, (int)world), "window grid");
  return sync(w);
}

eco_status eco_world_read_colours(eco_world* w, uint32_t world, float* out, size_t n_floats) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (world >= w->n_worlds || !out) return fail(ECO_EINVAL, "bad world or buffer");
  if (!w->L.colour) return fail(ECO_EINVAL, "the object has no colour trait (ECO_DESC_COLOUR_VISION)");
  const WorldParams& p = w->wp[world];
  if (n_floats < 3ull * p.cap) return fail(ECO_EINVAL, "colour buffer too small");
  std::vector<float> tmp(4ull * p.cap);
  std::vector<uint8_t> fl(p.cap);
  HIPCHK(w, hipMemcpyAsync(tmp.data(), w->d.colour + p.slot_off, 16ull * p.cap, hipMemcpyDeviceToHost, w->stream),
         "read colours");
  HIPCHK(w, hipMemcpyAsync(fl.data(), w->d.flags + p.slot_off, p.cap, hipMemcpyDeviceToHost, w->stream), "read flags");
  st = sync(w);
  if (st != ECO_OK) return st;
  for (size_t s = 0; s < p.cap; ++s)
    for (int k = 0; k < 3; ++k) out[3 * s + k] = (fl[s] & kAlive) ? tmp[4 * s + k] : NAN;
  return ECO_OK;
}

eco_status eco_world_write_colour(eco_world* w, uint32_t world, uint32_t slot, const float* rgb) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (world >= w->n_worlds || !rgb) return fail(ECO_EINVAL, "bad world or buffer");
  if (!w->L.colour) return fail(ECO_EINVAL, "the object has no colour trait (ECO_DESC_COLOUR_VISION)");
  const WorldParams& p = w->wp[world];
  if (slot >= p.cap) return fail(ECO_EINVAL, "slot out of range");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(rgb[k])) return fail(ECO_EINVAL, "colour must be finite");
  uint8_t fl = 0;
  HIPCHK(w, hipMemcpyAsync(&fl, w->d.flags + p.slot_off + slot, 1, hipMemcpyDeviceToHost, w->stream), "read flag");
  st = sync(w);
  if (st != ECO_OK) return st;
  if (!(fl & kAlive)) return fail(ECO_EINVAL, "slot not alive");
  const float4 c = make_float4(rgb[0], rgb[1], rgb[2], 0.0f);
  hipStream_t s = w->stream;
  HIPCHK(w, hipMemcpyAsync(w->d.colour + p.slot_off + slot, &c, 16, hipMemcpyHostToDevice, s), "write colour");
  HIPCHK(w, launch_render(s, w->d, w->ts, (int)world), "render");   // the window grid shows it from now on
  return sync(w);
}

eco_status eco_world_read_weights(eco_world* w, uint32_t world, uint32_t slot, int which, double* out, size_t n) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (world >= w->n_worlds || !out) return fail(ECO_EINVAL, "bad world or buffer");
  const WorldParams& p = w->wp[world];
  const Layout& L = w->L;
  if (slot >= p.cap) return fail(ECO_EINVAL, "slot out of range");
  if (n < L.P) return fail(ECO_EINVAL, "buffer too small");
  const uint64_t g = (uint64_t)p.slot_off + slot;
  const bool master = which == 1 || L.wdtype == ECO_W_FP32;
  std::vector<uint8_t> blk(master ? L.mstride : L.sstride);
  HIPCHK(w, hipMemcpyAsync(blk.data(), (master ? w->d.master + g * L.mstride : w->d.store + g * L.sstride), blk.size(),
                           hipMemcpyDeviceToHost, w->stream), "read weights");
  st = sync(w);
  if (st != ECO_OK) return st;
  for (uint32_t u = 0; u < L.u_end; ++u) {
    const HostUnit hu = host_unit(L, u);
    for (uint32_t i = 0; i < hu.nvalid; ++i) {
      double v;
      if (master) {
        float f;
        std::memcpy(&f, blk.data() + 16ull * u + 4 * i, 4);
        v = f;
      } else if (L.wdtype == ECO_W_BF16) {
        uint64_t off;
        if (hu.layer == 0) off = L.s_w1 + ((uint64_t)(hu.kb >> 1) * L.H1 + hu.row) * 16 + (hu.kb & 1) * 8;
        else if (hu.layer == 1) off = L.s_w2 + ((uint64_t)(hu.kb >> 1) * L.H2 + hu.row) * 16 + (hu.kb & 1) * 8;
        else if (hu.layer == 2) off = L.s_w3 + ((uint64_t)hu.row * L.H2 + 4 * hu.kb) * 2;
        else if (hu.layer == 3) off = L.s_b1 + (uint64_t)hu.row * 2;
        else if (hu.layer == 4) off = L.s_b2 + (uint64_t)hu.row * 2;
        else off = L.s_b3 + (uint64_t)hu.row * 2;
        uint16_t h;
        std::memcpy(&h, blk.data() + off + 2 * i, 2);
        v = host_bf16(h);
      } else {
        if (hu.layer >= 3) {
          const uint64_t off = (hu.layer == 3 ? L.s_b1 : (hu.layer == 4 ? L.s_b2 : L.s_b3)) + (uint64_t)hu.row * 4;
          float f;
          std::memcpy(&f, blk.data() + off + 4 * i, 4);
          v = f;
        } else {
          uint64_t off, soff;
          if (hu.layer == 0) { off = L.s_w1 + ((uint64_t)(hu.kb >> 2) * L.H1 + hu.row) * 16 + (hu.kb & 3) * 4; soff = L.s_sc1 + 4ull * hu.row; }
          else if (hu.layer == 1) { off = L.s_w2 + ((uint64_t)(hu.kb >> 2) * L.H2 + hu.row) * 16 + (hu.kb & 3) * 4; soff = L.s_sc2 + 4ull * hu.row; }
          else { off = L.s_w3 + (uint64_t)hu.row * L.H2 + 4 * hu.kb; soff = L.s_sc3 + 4ull * hu.row; }
          float sc;
          std::memcpy(&sc, blk.data() + soff, 4);
          v = host_fp8(blk[off + i]) * (double)sc;
        }
      }
      out[hu.p + i] = v;
    }
  }
  return ECO_OK;
}

eco_status eco_world_write_weights(eco_world* w, uint32_t world, uint32_t slot, const float* master, size_t n) {
  eco_status st = check_world(w);
  if (st != ECO_OK) return st;
  if (world >= w->n_worlds || !master) return fail(ECO_EINVAL, "bad world or buffer");
  const WorldParams& p = w->wp[world];
  const Layout& L = w->L;
  if (slot >= p.cap) return fail(ECO_EINVAL, "slot out of range");
  if (n < L.P) return fail(ECO_EINVAL, "buffer too small");
  std::vector<float> blk(L.mstride / 4, 0.0f);
  for (uint32_t u = 0; u < L.u_end; ++u) {
    const HostUnit hu = host_unit(L, u);
    for (uint32_t i = 0; i < hu.nvalid; ++i) blk[4ull * u + i] = master[hu.p + i];
  }
  const uint64_t g = (uint64_t)p.slot_off + slot;
  hipStream_t s = w->stream;
  HIPCHK(w, hipMemcpyAsync(w->d.master + g * L.mstride, blk.data(), 16ull * L.u_end, hipMemcpyHostToDevice, s),
         "write master");
  const uint32_t list[2] = {world, slot};
  HIPCHK(w, hipMemcpyAsync(w->emit_list, list, 8, hipMemcpyHostToDevice, s), "upload list");
  HIPCHK(w, launch_emit_list(s, w->d, L, w->emit_list, 1, EMIT_REQUANT, 0, 0, 0, 1), "requantise");
  st = sync(w);
  if (st != ECO_OK) return st;
  return ECO_OK;
}

eco_status eco_stream_read_gbps(void* hip_stream, uint64_t bytes, double* gbps) {
  if (!gbps) return fail(ECO_EINVAL, "gbps is NULL");
  bytes &= ~15ull;
  if (bytes < (64ull << 20)) return fail(ECO_EINVAL, "probe needs at least 64 MiB");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(ECO_EDEVICE, "no HIP device");
  void* buf = nullptr;
  uint32_t* sink = nullptr;
  if (hipMalloc(&buf, bytes) != hipSuccess) return fail(ECO_ENOMEM, "probe buffer");
  if (hipMalloc(&sink, 64) != hipSuccess) {
    (void)hipFree(buf);
    return fail(ECO_ENOMEM, "probe sink");
  }
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipMemsetAsync(buf, 0x5A, bytes, s);
  // a few grid shapes (blocks per CU x threads), best rate over five launches of each
  const uint32_t shapes[][2] = {{32, 256}, {64, 256}, {64, 512}};
  double best = 0.0;
  for (const auto& sh : shapes) {
    const uint32_t blocks = (uint32_t)cus * sh[0];
    if (e == hipSuccess) e = launch_stream_read(s, buf, bytes / 16, sink, blocks, sh[1]);  // warm-up
    for (int r = 0; r < 5 && e == hipSuccess; ++r) {
      e = hipEventRecord(a, s);
      if (e == hipSuccess) e = launch_stream_read(s, buf, bytes / 16, sink, blocks, sh[1]);
      if (e == hipSuccess) e = hipEventRecord(b, s);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e == hipSuccess && ms > 0.0f) best = std::max(best, (double)bytes / (ms * 1e-3) / 1e9);
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(sink);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(ECO_EDEVICE, hipGetErrorString(e));
  *gbps = best;
  return ECO_OK;
}

}  // extern "C"
