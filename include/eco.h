/*
 * eco.h -- C ABI of the MI355X (gfx950) world-step library libeco.so.
 *
 * The library advances one or more independent ecological worlds by whole
 * steps on the GPU.  One step is the transition of the paper's Ecological Game
 * (Sec. 3.1): every live agent observes the pre-step state through an
 * egocentric window plus scalar sensors (Sec. 3.2 "Sensors"), evaluates its own
 * MLP policy (Sec. 3.3), samples an action from the softmax, and the world then
 * applies turns, forward moves (one agent per cell; a contested empty cell goes
 * to the lowest slot), attacks where enabled (the victims' resources return to
 * their cells), eating, the per-step energy cost and death, single-parent
 * births directly behind the parent with Gaussian weight mutation into recycled
 * slots (Sec. 3.2 "Actions", Sec. 3.3), and resource regrowth (Sec. 3.2
 * "Resources").  The population function of Sec. 3.1 is exposed as the alive
 * flags and parent identities of the state.
 *
 * Conventions
 *  - Every call returns eco_status; the library never aborts or exits.
 *    eco_last_error() returns a thread-local message for the last failure.
 *  - Device buffers are owned by the eco_world (allocated through the caller's
 *    eco_allocator when one is given, else hipMalloc) and released by
 *    eco_world_destroy.  Host buffers passed in stay owned by the caller.
 *  - All work is enqueued on the stream given at create (NULL = the null
 *    stream).  eco_world_step is asynchronous; calls that return data to the
 *    host synchronise that stream first.
 *  - After a device error the object enters ECO_ESTATE: every call except
 *    reset/destroy/last_error fails until eco_world_reset succeeds.
 *  - An eco_world is not thread-safe; use one per host thread.
 *  - Energies are int32 fixed point in units of 0.1 energy.
 *  - Logical weight order (read/write_weights): W1[H1][D], b1[H1], W2[H2][H1],
 *    b2[H2], W3[A][H2], b3[A] (row = output unit), then the log temperature
 *    when it evolves (ECO_DESC_EVOLVE_TEMPERATURE).  The device layout is
 *    private.
 */
#ifndef ECO_H
#define ECO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eco_world eco_world;

typedef enum {
    ECO_OK = 0,
    ECO_EINVAL = -1,   /* bad argument / descriptor / buffer size */
    ECO_ENOMEM = -2,   /* device allocation failed */
    ECO_EDEVICE = -3,  /* a HIP call failed; the object is now in ECO_ESTATE */
    ECO_ESTATE = -4,   /* object unusable after an earlier device error */
    ECO_ENOTSUP = -5   /* valid but unsupported configuration */
} eco_status;

/* Storage format of the per-agent weights used by the forward pass.
 * FP32: the storage is the master copy.  BF16 (round-to-nearest-even) and
 * FP8 E4M3FN (OCP, per-output-row FP32 scale = row amax / 448, biases FP32)
 * are re-quantised from an FP32 master copy that mutation updates. */
typedef enum { ECO_W_FP32 = 0, ECO_W_BF16 = 1, ECO_W_FP8E4M3 = 2 } eco_wdtype;

/* Optional device allocator; alloc returns NULL on failure. */
typedef struct {
    void* (*alloc)(size_t bytes, void* ctx);
    void (*free)(void* ptr, void* ctx);
    void* ctx;
} eco_allocator;

/* Policy and sensor options (eco_world_desc.flags; identical for all worlds of
 * one object).
 *  ECO_DESC_FRONT_VISION: the S x S window lies ahead of the agent, which sits in
 *    the middle of the window's last row, instead of around it (App. "Varying
 *    Vision Range", "Front" configuration).
 *  ECO_DESC_EVOLVE_TEMPERATURE: every agent carries one more mutable parameter,
 *    theta_T, after the output biases; actions are drawn from the softmax of the
 *    logits divided by exp(theta_T) (Sec. 3.3).  theta_T starts at 0, is mutated
 *    like a weight and stored like a bias (BF16 in BF16 storage, FP32 otherwise).
 *  ECO_DESC_COLOUR_VISION: every agent carries a 3-channel colour trait, U[0,1)
 *    at init and the parent's plus mutation_sigma * N(0,1) per channel at birth;
 *    the window shows each cell as others see it (Sec. 3.2 "Sensors", Sec. 3.3):
 *    the occupant's colour, else green for a resource unit, grey for a wall,
 *    black; channels R, G, B = round(clamp(c, 0, 1) * 255) * 2^-8 and an
 *    elevation-difference channel, zero on the flat torus. */
#define ECO_DESC_FRONT_VISION 1u
#define ECO_DESC_EVOLVE_TEMPERATURE 2u
#define ECO_DESC_COLOUR_VISION 4u
/* ECO_DESC_ECOLOGY: the paper's three-resource ecology with health (Sec. 3.2
 * "Resources" and health points; App. "Varying Resource Rules", "Varying Agent
 * HP"), with the parameters of eco_world_desc.eco.  Cells hold water, energy and
 * biomass; agents carry the three in a capped stomach and have health.  Eight
 * actions: rest, turn left, turn right, forward, eat energy, eat water, eat
 * biomass, reproduce (n_actions = 8; with ECO_DESC_EVOLVE_TEMPERATURE the log
 * temperature follows the eight or nine output biases).  With
 * attack_enabled a ninth action, attack (index 8, n_actions = 9), strikes the
 * same 3x3 square as in the single-resource worlds, after the moves; an agent
 * on a cell struck k times loses k * attack_damage health in its health update
 * below (App. "Varying Attack Strength": full 100 = 10 HP, half 50, quarter 25),
 * and stats.killed counts the deaths of struck agents.  The attacker pays
 * e_cost_move.  Per live agent after the moves: the chosen resource
 * moves from its cell to its stomach (up to the eat amount, the cell's content and
 * the room under the cap); energy is spent (e_cost at rest, e_cost_move
 * otherwise; clamped at 0) and destroyed; w_cost water is spent onto the cell;
 * each resource that ran short costs hp_overspend health, age costs
 * age >> age_shift (and strikes as above); at health <= 0 the agent dies and its water, energy and
 * biomass go to its cell; otherwise, below full health, heal_energy energy buys
 * hp_heal health.  Reproduction (action 7) needs energy >= e_repro, water >=
 * w_child and biomass >= b_repro and gives the child e_child energy, w_child
 * water, b_child biomass and hp_child health.  Instead of regrowth, a cell with
 * biomass b below cell_energy_max energy gains one energy unit with probability
 * min(1, photo_rate * b) per step.  The window's four channels are agent present
 * and the cell's water, energy and biomass, each min(units, 255) * 2^-4; the
 * scalars (n_scalars 8, or 12 with the compass) are energy * 2^-8,
 * min(age, 1024) * 2^-10, water * 2^-8, biomass * 2^-3, health * 2^-7 and the own
 * cell's three channels.  Water and biomass are conserved.  With
 * ECO_DESC_COLOUR_VISION the window shows each cell as others see it instead:
 * the occupant's colour, else grey for a wall, else energy, biomass and water as
 * red, green, blue (min(16 e, 255), min(64 b, 255), min(16 w, 255)), each * 2^-8,
 * and the elevation difference (zero without terrain). */
#define ECO_DESC_ECOLOGY 8u
/* ECO_DESC_TERRAIN (with ECO_DESC_ECOLOGY; Sec. 3.2 "Terrain"): a rock height
 * 0..31 per cell, from a seeded value-noise field (lattice values
 * Philox(i + j*NX, 0, 9, 0).x0 >> 27 on an NX x NY torus lattice with
 * NX = max(1, width / terrain_scale), bilinear in exact integers with floor
 * division) or written with eco_world_write_terrain.  Water starts on the cells
 * below sea_level, (sea_level - rock) * water_per_depth units each (instead of
 * water sites), and at the end of every step all water on a cell moves to its
 * lowest 4-neighbour when that one lies strictly lower (the first of N, E, S, W
 * among equals), every cell at once.  With colour vision the window's fourth
 * channel is (rock(cell) - rock(agent's cell)) * 2^-3. */
#define ECO_DESC_TERRAIN 16u

/* Parameters of ECO_DESC_ECOLOGY (integer units; energy in 0.1 energy as the
 * e_* fields, health in 0.1 HP).  Initial cells: a water / energy / biomass site
 * with the given density holds water_site / energy_site / biomass_site units;
 * initial agents carry w_init water, b_init biomass and hp_max health. */
typedef struct {
    float water_density, energy_density, biomass_density;
    int32_t water_site, energy_site, biomass_site;
    int32_t eat_water, eat_biomass;              /* eat energy moves e_eat */
    int32_t cap_water, cap_energy, cap_biomass;  /* stomach capacities */
    int32_t e_cost_move, w_cost;
    float photo_rate;
    int32_t cell_energy_max;
    int32_t hp_max, hp_child, hp_overspend, hp_heal, heal_energy, age_shift;
    int32_t w_init, b_init, w_child, b_child, b_repro;
    int32_t terrain_scale, sea_level, water_per_depth;   /* ECO_DESC_TERRAIN */
    int32_t attack_damage;                       /* health per strike, 0..2^20 (attack_enabled) */
} eco_ecology;

/* One world (POD, copied at create).  Grid is a torus of width x height. */
typedef struct {
    uint32_t struct_size;        /* = sizeof(eco_world_desc) */
    uint32_t width, height;      /* 1 <= side, width*height < 2^31 */
    uint32_t n_agents_init;      /* agents placed at init (<= capacity, <= cells) */
    uint32_t capacity;           /* agent slots (births beyond it are blocked) */
    float resource_density;      /* initial P(cell holds one resource unit) */
    float regrow_prob;           /* per-step P(empty cell regrows one unit) */
    float mutation_sigma;        /* std of the child's Gaussian weight noise */
    uint32_t window;             /* S, odd, S <= width, S <= height, S <= 15 (ECO_ENOTSUP above) */
    uint32_t n_scalars;          /* 4 (internal+external) or 8 (+compass); ecology: 8 or 12 */
    uint32_t hidden1, hidden2;   /* each 32, 64 or 128 */
    uint32_t n_actions;          /* 5 (rest,L,R,fwd,eat) or 7 (+reproduce,+attack); ecology: 8, or 9
                                    with attack_enabled (+attack) */
    int32_t e_init, e_cost, e_eat, e_repro, e_child;  /* units of 0.1 energy; e_repro > 0 */
    uint32_t wdtype;             /* eco_wdtype; identical for all worlds of one object */
    uint32_t keep_master;        /* reserved: BF16/FP8 always keep an FP32 master */
    uint32_t attack_enabled;     /* 0: ATTACK does nothing; 1 (needs n_actions = 7; for the ecology,
                                    9 and the health damage described there): ATTACK kills
                                    every other agent in the 3x3 square directly ahead of the
                                    attacker (rows 1..3 ahead, one column to either side, torus),
                                    after the moves of the step; each victim leaves one resource
                                    unit on its cell (Sec. 3.2 actions and health points; App.
                                    "Varying Attack Strength", full strength) */
    uint32_t flags;              /* ECO_DESC_* (unknown bits: EINVAL) */
    eco_ecology eco;             /* used with ECO_DESC_ECOLOGY */
    uint64_t seed;               /* Philox key of this world */
} eco_world_desc;

/* Statistics of one step of one world (the measurement interface of App. E). */
typedef struct {
    uint64_t step;                     /* steps completed */
    uint64_t population;               /* live agents after the step */
    uint64_t births, deaths;           /* deaths: every death of the step, attacks included */
    uint64_t killed;                   /* agents killed by an attack this step (part of deaths) */
    uint64_t eaten, regrown;
    uint64_t moves_ok, moves_blocked;  /* FORWARD actions that did / did not move */
    uint64_t births_blocked_cell;      /* eligible parents whose cell behind was taken */
    uint64_t births_blocked_capacity;  /* winners left without a free slot */
    uint64_t resource_total;           /* resource units on the grid after regrowth */
    uint64_t action_hist[9];           /* actions taken by the agents live at step start */
    double energy_total;               /* sum of live energies (units of 0.1; exact) */
    double trait_mean, trait_var;      /* mean / variance over live agents of |theta_master|^2 */
    /* ECO_DESC_ECOLOGY (else 0): water and biomass on the grid and in live agents
       (both conserved), health of live agents.  There eaten counts eat actions
       that moved a unit, regrown the energy units photosynthesis added and
       resource_total the energy on the grid. */
    uint64_t water_total, biomass_total, hp_total;
} eco_stats;

/* Launch shape of the policy-forward kernel (tuned by eco_world_autotune). */
typedef struct {
    uint32_t waves_per_block;   /* 1, 2, 4 or 8 */
    uint32_t blocks_per_cu;     /* persistent grid = blocks_per_cu * CUs */
    uint32_t unroll;            /* 16-byte weight loads in flight per lane: 4, 8 or 16 */
    uint32_t reserved;
} eco_launch;

/* Static facts about an object (sizes for bandwidth accounting). */
typedef struct {
    uint32_t n_worlds, total_slots;
    uint64_t total_cells;
    uint32_t input_dim, hidden1, hidden2, n_actions;
    uint64_t param_count;              /* P */
    uint64_t weight_bytes_per_agent;   /* bytes one forward pass reads (algorithmic) */
    uint64_t storage_stride, master_stride;  /* device bytes per slot (0 = no master) */
    uint64_t device_bytes;             /* total device memory held */
    uint32_t n_cus;
    uint32_t wdtype;
} eco_info;

/* Per-kernel GPU time accumulated while ECO_RT_TIME_KERNELS is set.  REGROW runs
   fused into the BIRTH_CLAIM launch and SENSE (the per-cell window channels for
   the next step) into the COMPACT launch; both stay at zero. */
enum { ECO_K_FORWARD = 0, ECO_K_MOVE = 1, ECO_K_BIRTH_CLAIM = 2, ECO_K_BIRTH_SCAN = 3,
       ECO_K_BIRTH_COMMIT = 4, ECO_K_REGROW = 5, ECO_K_COMPACT = 6, ECO_K_SENSE = 7, ECO_K_COUNT = 8 };
typedef struct {
    double ms[8];
    uint64_t launches[8];
} eco_kernel_times;

/* Runtime flags (eco_world_set_flags). */
#define ECO_RT_KEEP_LOGITS 1u   /* forward writes FP32 logits for read_logits */
#define ECO_RT_USE_GRAPH 2u     /* eco_world_step replays captured hipGraphs of whole steps
                                   (default on): n steps as n / 32 replays of a 32-step graph
                                   and one graph of the remaining n mod 32 (each built on first
                                   use; the last four step counts are kept) */
#define ECO_RT_TIME_KERNELS 4u  /* hipEvents around every kernel group of eager launches; with
                                   ECO_RT_USE_GRAPH, event-record nodes around the policy kernel
                                   only, in a graph of the n steps of each eco_world_step call (one
                                   graph kept per n).  The call synchronises to read the times. */
#define ECO_RT_SPLIT_STEP 8u    /* an object of one world with at most 8,192
                                   slots and 16,384 cells, runs the step after the policy kernel
                                   as one fused launch (timed as ECO_K_MOVE); this flag runs the
                                   separate kernels instead.  Same integer state and statistics
                                   either way (the trait moments to rounding). */
/* The fused launch's limits: total slots and total cells of the object (each
 * world's ranges rounded up to 64). */
#define ECO_SMALL_STEP_MAX_SLOTS 8192u
#define ECO_SMALL_STEP_MAX_CELLS 16384u

/* Create n_worlds worlds (all with the same window, n_scalars, hidden sizes,
 * n_actions and wdtype) and run the deterministic init of Sec. 3.3 / placement.
 * hip_stream: a hipStream_t or NULL.  alloc: NULL = hipMalloc/hipFree.
 * descs[n_worlds] is copied (the caller keeps ownership); *out receives the new
 * object, owned by the caller until eco_world_destroy.  The object's device
 * memory comes from alloc (or hipMalloc) and stays with the object.
 * Errors: EINVAL (bad desc, with the field named; attack_enabled other than
 * 0/1, or 1 without n_actions = 7, 9 in the ecology), ENOTSUP (sizes without a
 * kernel), ENOMEM (an allocation returned NULL; what was allocated before it is
 * given back through alloc->free), EDEVICE (no current HIP device; with a
 * caller allocator this is found after allocating, and the memory is given
 * back).  *out is set to NULL first, so it is NULL after any error. */
eco_status eco_world_create(const eco_world_desc* descs, uint32_t n_worlds, void* hip_stream,
                            const eco_allocator* alloc, eco_world** out);
/* Wait for the object's stream, then release its graphs, events, streams and
 * device memory.  NULL is ignored. */
void eco_world_destroy(eco_world* w);
/* Text of the last error of the calling thread ("" if none); valid until the
 * thread's next failing call. */
const char* eco_last_error(void);

/* Advance every world by n_steps whole steps (asynchronous, except that
 * ECO_RT_TIME_KERNELS synchronises at the end to read its timers).  Under
 * ECO_RT_USE_GRAPH the first call with a step count captures the graphs it
 * replays (eco_world_prepare does that ahead of time). */
eco_status eco_world_step(eco_world* w, uint32_t n_steps);
/* Build, without running them, the graphs eco_world_step(w, n_steps) replays
 * under the current flags (the 32-step graph and the remainder's, or the timed
 * graph of n_steps), so the capture stays out of a caller's timed region.  No-op
 * without ECO_RT_USE_GRAPH or with n_steps = 0.  A later eco_world_set_flags,
 * eco_world_set_launch or eco_world_autotune drops the built graphs (after
 * waiting for the object's stream). */
eco_status eco_world_prepare(eco_world* w, uint32_t n_steps);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same n_steps steps
 * as eco_world_step, enqueued eagerly on the object's stream with no
 * allocation, no graph and no allocating library call.  The step's scratch
 * (tile partials, birth lists, step counters: about 8 bytes per slot plus
 * 128 bytes per 256-slot tile) lives in one static device array of 16 MiB per
 * GPU, held until the process ends; an object that needs more gets EINVAL and
 * nothing runs.  Every call on a GPU shares that GPU's array and nothing in it
 * has to start cleared; calls that overlap on one GPU (objects stepped on
 * different streams at once) race and must be serialised by the caller.
 * Returns like eco_world_step (asynchronous; ECO_RT_TIME_KERNELS and
 * ECO_RT_USE_GRAPH are ignored, ECO_RT_KEEP_LOGITS applies). */
eco_status eco_world_step_static(eco_world* w, uint32_t n_steps);

/* Re-initialise every world (the init of Sec. 3.3 and the placement of
 * Sec. 3.2: initial weights, positions, facings and resources, all from the
 * world's seed); seeds = NULL keeps each world's seed, else seeds[n_worlds]
 * replaces them.  Keeps the object's allocations and launch settings.  Clears
 * ECO_ESTATE on success; a device error leaves the object in ECO_ESTATE. */
eco_status eco_world_reset(eco_world* w, const uint64_t* seeds);

/* Latest step's statistics of worlds 0..min(n_worlds, max_worlds)-1 (synchronises). */
eco_status eco_world_stats(eco_world* w, eco_stats* out, uint32_t max_worlds);
/* The last up to max_records steps of one world, oldest first; *n_out = count.
 * The device ring keeps the most recent 1024 steps. */
eco_status eco_world_stats_history(eco_world* w, uint32_t world, eco_stats* out,
                                   uint32_t max_records, uint32_t* n_out);

/* Static facts of the object (sizes, bytes per agent; eco_info above). */
eco_status eco_world_info(const eco_world* w, eco_info* out);
/* Runtime flags (ECO_RT_*); unknown bits: EINVAL.  Drops the built graphs. */
eco_status eco_world_set_flags(eco_world* w, uint32_t flags);
/* Policy-kernel launch shape; shapes outside the documented ranges: EINVAL.
 * Every shape gives bit-identical results.  Drops the built graphs. */
eco_status eco_world_set_launch(eco_world* w, const eco_launch* launch);
eco_status eco_world_get_launch(const eco_world* w, eco_launch* out);
/* Time every candidate launch shape on the forward pass of the current state
 * (the forward has no side effect on the world) in nine rounds over all shapes
 * (median per shape), then the four fastest again as runs of three launches in
 * eleven rounds, and keep the shape with the lowest mean of the second pass.
 * Every candidate produces bit-identical actions.  *best may be NULL. */
eco_status eco_world_autotune(eco_world* w, eco_launch* best);
/* eco_world_autotune with a persistent result cache: a text file of JSON lines
 * {"key": ..., "waves_per_block": .., "blocks_per_cu": .., "unroll": .., "ms": ..}.
 * The key names what the choice depends on: the device architecture and CU
 * count, the policy shape (D, H, A, window, storage type, window words, ninth
 * row) and the live population rounded to a power of two.  A line with this
 * object's key sets the launch without timing anything (*from_cache = 1);
 * otherwise the shapes are timed as above and a line is appended (*from_cache
 * = 0; a file that cannot be written is not an error).  path NULL: EINVAL.
 * best and from_cache may be NULL. */
eco_status eco_world_autotune_cached(eco_world* w, const char* path, eco_launch* best, int* from_cache);
/* Accumulated per-kernel-group times of the steps run with ECO_RT_TIME_KERNELS
 * (milliseconds and launch counts); reset != 0 zeroes them after reading. */
eco_status eco_world_kernel_times(eco_world* w, eco_kernel_times* out, int reset);

/* Measurement helper, not part of the step: the device's streaming-read rate.
 * Allocates `bytes` of device memory (hipMalloc; rounded down to 16 B, at least
 * 64 MiB), fills it, times five launches each of a kernel that reads it once
 * with 16-byte non-temporal loads (grid-stride, 8 loads in flight per lane) at
 * three grid shapes, frees it, and writes the best rate in GB/s (1e9 B/s) to *gbps.  hip_stream
 * may be NULL (the default stream).  Errors: EINVAL (null gbps or too small),
 * ENOMEM, EDEVICE. */
eco_status eco_stream_read_gbps(void* hip_stream, uint64_t bytes, double* gbps);

/* ---- parity / test hooks (not on the timed path) ------------------------ */

/* One step with the given actions (host array, one per slot of every world,
 * worlds concatenated in order; entries of dead slots ignored; values must be
 * < n_actions for live slots).  The policy still runs, so read_logits and
 * read_sampled report what the policy would have done. */
eco_status eco_world_step_with_actions(eco_world* w, const uint8_t* actions);

/* Integer state of one world, layout (little endian):
 *   u64 step, u64 uid_next, u32 width, u32 height, u32 capacity, u32 0   (32 B)
 *   u64 uid[cap], u64 parent_uid[cap], i32 pos[cap], i32 energy[cap], i32 age[cap],
 *   i32 occ[cells], u8 facing[cap], u8 alive[cap], u8 action[cap], u8 res[cells], u8 wall[cells]
 *   then with ECO_DESC_ECOLOGY: i32 water[cap], i32 biomass[cap], i32 hp[cap],
 *   i32 cell_water[cells], i32 cell_energy[cells], i32 cell_biomass[cells]
 * pos = y*width + x; occ = slot or -1; facing 0..3 = N,E,S,W (y grows down);
 * parent_uid of initial agents = UINT64_MAX.  Fields of dead slots other than
 * alive are unspecified.  bytes must be >= eco_world_state_bytes(). */
size_t eco_world_state_bytes(const eco_world* w, uint32_t world);
eco_status eco_world_read_state(eco_world* w, uint32_t world, void* buf, size_t bytes);
/* Replace the integer state; slots alive in buf but not before get the
 * initial weights of their slot index.  Must keep occ consistent with pos;
 * res and wall hold 0 or 1 per cell (ECO_EINVAL otherwise). */
eco_status eco_world_write_state(eco_world* w, uint32_t world, const void* buf, size_t bytes);

/* FP32 logits of the last step's forward, [cap][n_actions]; NaN for slots not
 * live at that step's start.  Requires ECO_RT_KEEP_LOGITS during that step. */
eco_status eco_world_read_logits(eco_world* w, uint32_t world, float* out, size_t n_floats);
/* The policy's sampled action of the last step per slot (255 if not live). */
eco_status eco_world_read_sampled(eco_world* w, uint32_t world, uint8_t* out, size_t n);

/* The rock layer of one world (ECO_DESC_TERRAIN objects only, else EINVAL):
 * rock[width * height] heights 0..31.  Writing it recomputes the flow
 * directions and the window grid; the water stays where it is. */
eco_status eco_world_read_terrain(eco_world* w, uint32_t world, int32_t* rock, size_t n);
eco_status eco_world_write_terrain(eco_world* w, uint32_t world, const int32_t* rock, size_t n);

/* Colour traits of one world (ECO_DESC_COLOUR_VISION objects only, else EINVAL):
 * out[cap][3] FP32 R, G, B; NaN for slots not alive.  n_floats >= 3 * capacity. */
eco_status eco_world_read_colours(eco_world* w, uint32_t world, float* out, size_t n_floats);
/* Overwrite the colour of live slot `slot` (finite values; EINVAL otherwise) and
 * re-render that world's window grid, so the next step's observations show it. */
eco_status eco_world_write_colour(eco_world* w, uint32_t world, uint32_t slot, const float* rgb);

/* Weights of one live slot in logical order as doubles: which = 0 the storage
 * values dequantised exactly, which = 1 the FP32 master. */
eco_status eco_world_read_weights(eco_world* w, uint32_t world, uint32_t slot, int which,
                                  double* out, size_t n);
/* Overwrite one slot's FP32 master (logical order) and re-quantise its storage. */
eco_status eco_world_write_weights(eco_world* w, uint32_t world, uint32_t slot,
                                   const float* master, size_t n);

#ifdef __cplusplus
}
#endif
#endif /* ECO_H */
