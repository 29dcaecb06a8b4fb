/*
 * eco_oracle.h -- CPU oracle for the ecological world step (TEST INFRASTRUCTURE).
 *
 * This is a plain, slow, sequential implementation of one world step of the
 * paper's Ecological Game (Sec. 3.1: transition + population function +
 * observation function; Sec. 3.2: resources, sensors, actions, reproduction;
 * Sec. 3.3: per-agent MLP policy, softmax sampling, Gaussian mutation), in FP64
 * for the policy and exact integers for the world.  It shares no code, header,
 * table or constant with the GPU library; only tests/, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  The product path never calls it.
 *
 * Every function follows the step algorithm written out in eco_oracle.c, whose
 * comments cite the passage of the paper each rule restates.
 */
#ifndef ECO_ORACLE_H
#define ECO_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Weight storage formats the oracle evaluates logits on. */
enum { ORC_FP32 = 0, ORC_BF16 = 1, ORC_FP8 = 2 };

/* Actions.  A = 5 uses 0..4; A = 7 adds REPRODUCE and ATTACK (ATTACK does
 * nothing unless the world has attack_enabled).  The ecology's eight or nine
 * actions follow below. */
enum { ORC_REST = 0, ORC_TURN_L = 1, ORC_TURN_R = 2, ORC_FORWARD = 3, ORC_EAT = 4,
       ORC_REPRODUCE = 5, ORC_ATTACK = 6 };

/* Policy and sensor options (orc_desc.flags).
 *   ORC_FRONT_VISION: the S x S window lies ahead of the agent, which sits in the
 *     middle of its last row, instead of around it (App. "Varying Vision Range").
 *   ORC_EVOLVE_TEMPERATURE: every agent carries one more mutable parameter, its
 *     log softmax temperature, after the output biases (Sec. 3.3).
 *   ORC_COLOUR_VISION: every agent carries a 3-channel colour trait that mutates
 *     like its weights, and the window shows the rendered colour of each cell
 *     plus an elevation-difference channel (zero on the flat torus) (Sec. 3.2
 *     "Sensors", Sec. 3.3). */
enum { ORC_FRONT_VISION = 1, ORC_EVOLVE_TEMPERATURE = 2, ORC_COLOUR_VISION = 4, ORC_ECOLOGY = 8, ORC_TERRAIN = 16 };

/* ORC_TERRAIN (with ORC_ECOLOGY): a rock layer of heights 0..31 (Sec. 3.2
 * "Terrain"), from a seeded value-noise field (lattice spacing terrain_scale,
 * bilinear in exact integers) or written by the caller; water starts on the
 * cells below sea_level, (sea_level - rock) * water_per_depth units each, and
 * every step all water on a cell moves to its lowest 4-neighbour when that one
 * lies strictly lower (ties: N, E, S, W), all cells at once.  With colour vision
 * the window's fourth channel is the elevation difference to the agent's cell. */

/* ORC_ECOLOGY: the paper's three-resource ecology with health (Sec. 3.2
 * "Resources" and health points; App. "Varying Resource Rules", "Varying Agent
 * HP").  Cells hold water, energy and biomass; agents carry the three in a
 * capped stomach plus health.  Eight actions: rest, turn left, turn right,
 * forward, eat energy, eat water, eat biomass, reproduce (and attack, with
 * attack_enabled).  Amounts are integer
 * units: energies in 0.1 energy (as e_*), health in 0.1 HP. */
enum { ORC_EAT_ENERGY = 4, ORC_EAT_WATER = 5, ORC_EAT_BIOMASS = 6, ORC_REPRODUCE_ECO = 7, ORC_ATTACK_ECO = 8 };
/* With attack_enabled the ecology has a ninth action, ORC_ATTACK_ECO: it strikes
 * the same 3x3 square ahead as ORC_ATTACK, and every struck agent loses
 * attack_damage health per attacker that struck its cell, in the same health
 * update as its overspend and age damage (App. "Varying Attack Strength": full
 * strength 10 HP = 100 units kills any agent of full health, half 50, quarter
 * 25). */
typedef struct {
    float    water_density, energy_density, biomass_density;  /* initial site densities */
    int32_t  water_site, energy_site, biomass_site;            /* units on an initial site */
    int32_t  eat_water, eat_biomass;                           /* units one eat moves (energy: e_eat) */
    int32_t  cap_water, cap_energy, cap_biomass;               /* stomach capacities */
    int32_t  e_cost_move;                                      /* energy cost of any action but rest (rest: e_cost) */
    int32_t  w_cost;                                           /* water spent per step, returned to the cell */
    float    photo_rate;                                       /* energy units per biomass unit per step */
    int32_t  cell_energy_max;                                  /* photosynthesis fills a cell up to this */
    int32_t  hp_max, hp_child;                                 /* health at init / at birth */
    int32_t  hp_overspend;                                     /* damage per step per overspent resource */
    int32_t  hp_heal, heal_energy;                             /* health gained / energy paid per healing step */
    int32_t  age_shift;                                        /* age damage per step = age >> age_shift */
    int32_t  w_init, b_init;                                   /* initial agents' water and biomass */
    int32_t  w_child, b_child, b_repro;                        /* given to a child; biomass needed to reproduce */
    int32_t  terrain_scale, sea_level, water_per_depth;        /* ORC_TERRAIN */
    int32_t  attack_damage;                                    /* health per strike (with attack_enabled) */
} orc_ecology;

/* One world's parameters.  Energies are integers in units of 0.1 energy. */
typedef struct {
    uint32_t width, height;            /* toroidal grid */
    uint32_t n_agents_init, capacity;  /* initial live agents, slot capacity */
    float    resource_density;         /* initial Bernoulli density of resource cells */
    float    regrow_prob;              /* per-step regrowth probability of an empty cell */
    float    mutation_sigma;           /* std of the Gaussian mutation noise */
    uint32_t window;                   /* S, odd */
    uint32_t n_scalars;                /* 4 or 8 */
    uint32_t hidden1, hidden2, n_actions;
    int32_t  e_init, e_cost, e_eat, e_repro, e_child;
    uint32_t wdtype;                   /* ORC_FP32 / ORC_BF16 / ORC_FP8 */
    uint32_t attack_enabled;           /* 0 or 1; 1 needs n_actions == 7 (ecology: 9) */
    uint32_t flags;                    /* ORC_FRONT_VISION | ORC_EVOLVE_TEMPERATURE | ORC_COLOUR_VISION | ORC_ECOLOGY | ORC_TERRAIN */
    orc_ecology eco;                   /* used with ORC_ECOLOGY */
    uint64_t seed;
} orc_desc;

/* Per-step statistics (the measurement interface of App. E).  deaths counts
 * every death of the step; killed is the part of it caused by attacks (in the
 * ecology: the deaths of agents struck this step).  With
 * ORC_ECOLOGY: eaten counts eat actions that moved a unit, regrown the energy
 * units photosynthesis added, resource_total the energy on the grid, and
 * water_total / biomass_total the water and biomass on the grid and in live
 * agents (both conserved), hp_total the health of live agents; else 0. */
typedef struct {
    uint64_t step, population, births, deaths, killed, eaten, regrown, moves_ok, moves_blocked,
             births_blocked_cell, births_blocked_capacity, resource_total, action_hist[9];
    double   energy_total, trait_mean, trait_var;
    uint64_t water_total, biomass_total, hp_total;
} orc_stats;

typedef struct orc_world orc_world;

/* Sizes derived from a desc: D = 4*S*S + n_s inputs, P parameters (the network's,
 * plus the log temperature when it evolves). */
uint32_t orc_input_dim(const orc_desc* d);
uint64_t orc_param_count(const orc_desc* d);

/* Create a world and run the deterministic init.  materialize != 0 keeps every
 * live agent's weights in memory (needed to sample actions).  materialize == 0
 * ("lineage mode", for full-size worlds driven by given actions) keeps only each
 * agent's lineage (root slot + the (parent slot, step) of every mutation):
 * weights are rebuilt on demand for sampled agents and the trait statistics are
 * NaN.  Returns NULL on invalid desc (orc_last_error() says why). */
orc_world* orc_create(const orc_desc* d, int materialize);
void       orc_destroy(orc_world* w);
const char* orc_last_error(void);

/* One step.  actions: NULL = sample from the policy, else one action per slot
 * (entries of dead slots are ignored).  logits_out: NULL or [capacity][A] (NaN
 * for slots not live at step start).  sampled_out: NULL or [capacity] (the
 * policy's own choice; 255 for dead slots; needs materialized weights).
 * Returns 0, or -1 with orc_last_error(). */
int orc_step(orc_world* w, const uint8_t* actions, double* logits_out, uint8_t* sampled_out);

/* Logits of live slot `slot` on the current state, FP64 (materialized or lineage). */
int orc_agent_logits(orc_world* w, uint32_t slot, double* out /* [A] */);

/* The FP64 observation vector x (D values) of live slot `slot`. */
int orc_observe(const orc_world* w, uint32_t slot, double* out /* [D] */);

/* Weights of live slot `slot` in logical nn.Linear order
 * (W1[H1][D], b1, W2[H2][H1], b2, W3[A][H2], b3, then the log temperature when
 * it evolves).
 * which = 0: storage values dequantised exactly (FP32 = master), 1: FP32 master. */
int orc_read_weights(orc_world* w, uint32_t slot, int which, double* out /* [P] */);

/* State access.  State byte layout (shared by interface contract with the
 * library's read_state, written independently here):
 *   u64 step, u64 uid_next, u32 width, u32 height, u32 capacity, u32 reserved  (32 B)
 *   u64 uid[cap], u64 parent_uid[cap], i32 pos[cap], i32 energy[cap], i32 age[cap],
 *   i32 occ[cells], u8 facing[cap], u8 alive[cap], u8 action[cap], u8 res[cells],
 *   u8 wall[cells]
 *   then with ORC_ECOLOGY: i32 water[cap], i32 biomass[cap], i32 hp[cap],
 *   i32 cell_water[cells], i32 cell_energy[cells], i32 cell_biomass[cells]
 * pos = y*width + x. */
size_t orc_state_bytes(const orc_world* w);
int    orc_read_state(const orc_world* w, void* buf, size_t bytes);
/* Overwrite the integer state.  Newly alive slots get fresh initial weights for
 * that slot index (as at init); trait is recomputed. */
int    orc_write_state(orc_world* w, const void* buf, size_t bytes);

int orc_stats_get(const orc_world* w, orc_stats* out);

/* The rock layer (ORC_TERRAIN): read, or overwrite (heights 0..31; the flow
 * directions follow; the water stays where it is). */
int orc_read_terrain(const orc_world* w, int32_t* rock /* [cells] */);
int orc_write_terrain(orc_world* w, const int32_t* rock);

/* Colour trait of live slot `slot` (FP32 R, G, B), and its overwrite. */
int orc_read_colour(const orc_world* w, uint32_t slot, float out[3]);
int orc_write_colour(orc_world* w, uint32_t slot, const float in[3]);

/* Building blocks exposed for the pins. */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void   orc_gauss4(const uint32_t ctr[4], const uint32_t key[2], double z[4]);
void   orc_cos_sin_2pi_u24(uint32_t j, double cs[2]);   /* cos, sin of 2 pi j 2^-24 */
uint16_t orc_bf16_rne(float x);
uint8_t  orc_fp8e4m3_rne_sat(float x);
double   orc_fp8e4m3_decode(uint8_t q);
/* Inverse-CDF softmax sample of A logits with uniform u in [0,1); the tempered
 * form divides the logits by exp(log_tau). */
int    orc_sample(const double* logits, int A, double u);
int    orc_sample_tempered(const double* logits, int A, double log_tau, double u);
/* The 8-bit rendering of one colour channel: round(clamp(c, 0, 1) * 255), ties up. */
uint32_t orc_colour_byte(float c);

#ifdef __cplusplus
}
#endif
#endif
