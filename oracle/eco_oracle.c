/*
 * eco_oracle.c -- CPU oracle for the ecological world step.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, sequential, slow on purpose: one loop per
 * rule, FP64 for the policy, exact integers for the world.  Shares no code with
 * the GPU library (see eco_oracle.h).
 *
 * What it computes, and where the paper states it:
 *   - The state is factored into map layers and per-agent records (Sec. 3.2).
 *     Map: occupancy (one agent per cell), one resource layer, a static wall
 *     mask.  Agent: position, facing, energy, age, identity and parent
 *     identity (the population function of Sec. 3.1 reads alive + parent uid).
 *   - Observation (Sec. 3.2 "Sensors"; App. F vision layout): an egocentric
 *     S x S window drawn with the agent facing the top of the page ("Around"
 *     layout), 4 channels per cell, then internal/external/compass scalars.
 *   - Policy (Sec. 3.3): per-agent memoryless MLP with two ReLU hidden layers
 *     and a linear head; actions drawn from the softmax (temperature 1).
 *   - Actions (Sec. 3.2 "Actions"): rest, rotate CCW/CW, forward, eat,
 *     reproduce, attack.  Contested or occupied targets do not move; here the
 *     lowest slot wins a contested empty cell.  With attacks enabled (the "+A"
 *     worlds), an attack kills every other agent in the 3x3 square of cells
 *     directly ahead of the attacker; a dead agent's carried resource returns
 *     to its cell (Sec. 3.2, health points; App. "Varying Attack Strength", full
 *     strength).  In the ecology the attack is the ninth action and each strike
 *     costs the struck agent a set amount of health (full, half or quarter
 *     strength).
 *   - Resources (Sec. 3.2 "Resources"): every step costs energy, eating moves a
 *     resource unit from the cell into the agent, energy slowly regrows on
 *     empty cells (Bernoulli per cell and step).
 *   - The three-resource ecology (ORC_ECOLOGY; Sec. 3.2 "Resources" and health
 *     points; App. "Varying Resource Rules", "Varying Agent HP"): water, energy
 *     and biomass on the grid and in capped stomachs, three eat actions, every
 *     action spends energy (least for rest, destroyed) and water (returned to
 *     the cell), overspending and age damage health, energy heals it, death at
 *     zero health returns everything carried to the cell, reproduction needs
 *     spare biomass, energy grows on free-standing biomass (photosynthesis).
 *   - Terrain (ORC_TERRAIN; Sec. 3.2 "Terrain"): a rock height per cell, water
 *     first filling the cells below sea level, then flowing downhill every step
 *     by a discrete rule; vision shows the local elevation difference.
 *   - Reproduction (Sec. 3.2 "Actions", Sec. 3.3): single parent with enough
 *     energy, child placed directly behind the parent, child receives a fixed
 *     amount of the parent's energy, child weights = parent weights + Gaussian
 *     noise on every mutable value.  Initial weights are Gaussian with zero
 *     biases (Sec. 3.3; here N(0, 1/fan_in)).
 *
 * Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11), keyed by the world seed, with
 * counter (entity, step, stream, block).  Gaussians use the Box-Muller
 * transform (Box & Muller, 1958) with libm log/cos/sin/sqrt in FP64.
 */
#include "eco_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* errors                                                                    */
/* ------------------------------------------------------------------------- */
static _Thread_local char g_err[256] = "";
static int fail(const char* msg) { snprintf(g_err, sizeof g_err, "%s", msg); return -1; }
const char* orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (SC'11): 10 rounds of two 32x32->64 multiplies; the key is   */
/* bumped by the Weyl constants between rounds.                               */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream tags of the counter's third word. */
enum { ST_CELLKEY = 0, ST_FACING = 1, ST_RESINIT = 2, ST_WINIT = 3, ST_ACTION = 4,
       ST_MUTATE = 5, ST_REGROW = 6, ST_COLOUR_INIT = 7, ST_COLOUR_MUTATE = 8, ST_TERRAIN = 9 };

static uint32_t draw_x0(const uint32_t key[2], uint32_t a, uint32_t step, uint32_t stream, uint32_t blk) {
    uint32_t ctr[4] = {a, step, stream, blk}, out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[0];
}

/* The regrowth (or photosynthesis) draw of cell c at step t: output c mod 4 of
 * the block with counter (c / 4, t, REGROW, 0), one block for four neighbouring
 * cells, as a parameter takes output p mod 4 of its mutation block. */
static uint32_t draw_cell(const uint32_t key[2], uint32_t c, uint32_t step) {
    uint32_t ctr[4] = {c >> 2, step, ST_REGROW, 0}, out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[c & 3];
}

/* cos and sin of 2 pi j 2^-24 for 0 <= j < 2^24.  The whole quarter turns
 * q = j >> 22 come off exactly; of the rest r (a fraction r 2^-22 of a quarter
 * turn) libm gets the angle from the nearer end of the quarter, 2 pi r 2^-24 or
 * its complement 2 pi (2^22 - r) 2^-24 (swapping cos and sin), so every
 * argument lies in [0, pi/4], where cos and sin keep their relative accuracy,
 * and the zeros at the quarter turns are exact. */
void orc_cos_sin_2pi_u24(uint32_t j, double cs[2]) {
    const double two_pi = 6.283185307179586476925286766559;
    const uint32_t q = (j >> 22) & 3u, r = j & 0x3FFFFFu;
    double c, s;
    if (r <= 0x200000u) {
        const double th = two_pi * (double)r * 0x1p-24;
        c = cos(th);
        s = sin(th);
    } else {
        const double th = two_pi * (double)(0x400000u - r) * 0x1p-24;
        c = sin(th);
        s = cos(th);
    }
    /* a quarter turn maps (cos, sin) to (-sin, cos) */
    cs[0] = q == 0 ? c : (q == 1 ? -s : (q == 2 ? -c : s));
    cs[1] = q == 0 ? s : (q == 1 ? c : (q == 2 ? -s : -c));
}

/* Box-Muller on one Philox block: (x0,x1) -> z0,z1 and (x2,x3) -> z2,z3.
 * u1 = ((x>>8)+1) 2^-24 lies in (0,1] so log(u1) is finite; u2 = (y>>8) 2^-24,
 * and z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2). */
void orc_gauss4(const uint32_t ctr[4], const uint32_t key[2], double z[4]) {
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    for (int pair = 0; pair < 2; ++pair) {
        double u1 = (double)((x[2 * pair] >> 8) + 1u) * 0x1p-24;
        double r = sqrt(-2.0 * log(u1));
        double cs[2];
        orc_cos_sin_2pi_u24(x[2 * pair + 1] >> 8, cs);
        z[2 * pair] = r * cs[0];
        z[2 * pair + 1] = r * cs[1];
    }
}

/* Integer threshold for a Bernoulli(p) draw on a 32-bit uniform: x < floor(p 2^32). */
static uint64_t bern_threshold(float p) {
    double t = floor((double)p * 4294967296.0);
    if (t < 0) t = 0;
    if (t > 4294967296.0) t = 4294967296.0;
    return (uint64_t)t;
}

/* ------------------------------------------------------------------------- */
/* Number formats                                                            */
/* ------------------------------------------------------------------------- */
/* bfloat16 round-to-nearest-even of a finite float: add half an ulp of the
 * kept part (0x7FFF plus the kept LSB for ties) and truncate. */
uint16_t orc_bf16_rne(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}
static double bf16_value(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* OCP FP8 E4M3FN: sign, 4 exponent bits (bias 7), 3 mantissa bits, no
 * infinities, 0x7F/0xFF are NaN, largest finite 448. */
double orc_fp8e4m3_decode(uint8_t q) {
    int s = q >> 7, e = (q >> 3) & 15, m = q & 7;
    if (e == 15 && m == 7) return NAN;
    double v = (e == 0) ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, e - 7);
    return s ? -v : v;
}
/* Round to nearest, ties to even code, saturating at 448: a binary search for
 * the two neighbouring non-negative codes (value is monotone in the code). */
uint8_t orc_fp8e4m3_rne_sat(float x) {
    uint8_t sign = (x < 0.0f) ? 0x80 : 0x00;
    double a = fabs((double)x);
    if (a >= 448.0) return (uint8_t)(sign | 0x7E);
    int lo = 0, hi = 0x7E;                 /* decode(lo) <= a < decode(hi) */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (orc_fp8e4m3_decode((uint8_t)mid) <= a) lo = mid; else hi = mid;
    }
    double dlo = a - orc_fp8e4m3_decode((uint8_t)lo), dhi = orc_fp8e4m3_decode((uint8_t)hi) - a;
    int q = (dlo < dhi) ? lo : (dhi < dlo) ? hi : ((lo & 1) ? hi : lo);
    if (q == 0) return 0;                  /* +0 for tiny values of either sign */
    return (uint8_t)(sign | q);
}

/* ------------------------------------------------------------------------- */
/* World                                                                     */
/* ------------------------------------------------------------------------- */
typedef struct { int64_t parent; uint32_t parent_slot; uint32_t step; uint32_t root; } lineage_node;

struct orc_world {
    orc_desc d;
    uint32_t W, H, cells, cap, S, R, ns, D, H1, H2, A;
    uint64_t P;
    uint32_t key[2];
    uint64_t step, uid_next;
    int32_t *pos, *energy, *age;
    uint8_t *facing, *alive, *action;
    uint64_t *uid, *puid;
    int32_t *occ;
    uint8_t *res, *wall;
    int materialize;
    float *master;            /* [cap][P] FP32 master, materialized mode */
    double *stored;           /* [cap][P] dequantised storage (BF16/FP8), materialized mode */
    int64_t *node;            /* [cap] lineage node of each live slot */
    lineage_node *nodes;
    size_t n_nodes, nodes_cap;
    double *trait;            /* [cap] squared L2 norm of the FP32 master */
    float *colour;            /* [cap][3] colour trait (colour vision only; kept in lineage mode too,
                                 since every observation renders the occupants' colours) */
    int eco;                  /* ORC_ECOLOGY */
    int32_t *water, *biomass, *hp;      /* [cap] stomach water and biomass, health (ecology) */
    int32_t *cw, *ce, *cb;              /* [cells] water, energy, biomass on the grid (ecology) */
    int32_t *rock;                      /* [cells] terrain heights 0..31 (ORC_TERRAIN) */
    int8_t *flowdir;                    /* [cells] direction water leaves by, -1 = it stays (ORC_TERRAIN) */
    orc_stats stats;
};

uint32_t orc_input_dim(const orc_desc* d) { return 4u * d->window * d->window + d->n_scalars; }
uint64_t orc_param_count(const orc_desc* d) {
    uint64_t D = orc_input_dim(d), H1 = d->hidden1, H2 = d->hidden2, A = d->n_actions;
    uint64_t net = D * H1 + H1 + H1 * H2 + H2 + H2 * A + A;
    return net + ((d->flags & ORC_EVOLVE_TEMPERATURE) ? 1u : 0u);   /* + the log temperature */
}

/* Facing 0..3 = N, E, S, W; y grows downward. */
static const int DX[4] = {0, 1, 0, -1};
static const int DY[4] = {-1, 0, 1, 0};

static uint32_t wrap_cell(const orc_world* w, int64_t x, int64_t y) {
    int64_t xx = ((x % (int64_t)w->W) + (int64_t)w->W) % (int64_t)w->W;
    int64_t yy = ((y % (int64_t)w->H) + (int64_t)w->H) % (int64_t)w->H;
    return (uint32_t)(yy * (int64_t)w->W + xx);
}
static uint32_t step_cell(const orc_world* w, uint32_t cell, int facing, int sign) {
    int64_t x = cell % w->W, y = cell / w->W;
    return wrap_cell(w, x + sign * DX[facing], y + sign * DY[facing]);
}

/* Layer geometry in the logical parameter vector. */
typedef struct { uint64_t w_off, b_off; uint32_t rows, cols; } layer_geom;
static void layers(const orc_world* w, layer_geom L[3]) {
    uint64_t o = 0;
    L[0].rows = w->H1; L[0].cols = w->D;  L[0].w_off = o; o += (uint64_t)w->H1 * w->D;  L[0].b_off = o; o += w->H1;
    L[1].rows = w->H2; L[1].cols = w->H1; L[1].w_off = o; o += (uint64_t)w->H2 * w->H1; L[1].b_off = o; o += w->H2;
    L[2].rows = w->A;  L[2].cols = w->H2; L[2].w_off = o; o += (uint64_t)w->A * w->H2;  L[2].b_off = o; o += w->A;
}

/* Initial weights of slot j: N(0, 1/fan_in) weights, zero biases, and a zero log
 * temperature (temperature 1) when it evolves.  The Gaussian for logical
 * parameter p is output p%4 of block p/4 of stream WINIT. */
static void init_weights(const orc_world* w, uint32_t j, float* out) {
    layer_geom L[3];
    layers(w, L);
    double z[4];
    uint64_t cur_blk = UINT64_MAX;
    for (int l = 0; l < 3; ++l) {
        double std = sqrt(1.0 / (double)L[l].cols);
        uint64_t nw = (uint64_t)L[l].rows * L[l].cols;
        for (uint64_t i = 0; i < nw; ++i) {
            uint64_t p = L[l].w_off + i;
            if (p / 4 != cur_blk) {
                cur_blk = p / 4;
                uint32_t ctr[4] = {j, 0u, ST_WINIT, (uint32_t)cur_blk};
                orc_gauss4(ctr, w->key, z);
            }
            out[p] = (float)(z[p % 4] * std);
        }
        for (uint32_t r = 0; r < L[l].rows; ++r) out[L[l].b_off + r] = 0.0f;
    }
    if (w->d.flags & ORC_EVOLVE_TEMPERATURE) out[w->P - 1] = 0.0f;
}

/* Initial colour of slot j: three uniforms in [0, 1) from one Philox block,
 * c_k = (x_k >> 8) 2^-24 (exact in FP32). */
static void init_colour(const orc_world* w, uint32_t j, float* c) {
    uint32_t ctr[4] = {j, 0u, ST_COLOUR_INIT, 0u}, x[4];
    orc_philox4x32_10(ctr, w->key, x);
    for (int k = 0; k < 3; ++k) c[k] = (float)((double)(x[k] >> 8) * 0x1p-24);
}

/* The child's colour: the parent's plus sigma times a Gaussian per channel (the
 * first three of one Box-Muller block), rounded like the weights. */
static void mutate_colour(const orc_world* w, const float* parent, uint32_t parent_slot, uint32_t step, float* child) {
    uint32_t ctr[4] = {parent_slot, step, ST_COLOUR_MUTATE, 0u};
    double z[4];
    orc_gauss4(ctr, w->key, z);
    for (int k = 0; k < 3; ++k) child[k] = (float)fma((double)w->d.mutation_sigma, z[k], (double)parent[k]);
}

uint32_t orc_colour_byte(float c) {
    double x = (double)c;
    if (!(x > 0.0)) x = 0.0;
    if (x > 1.0) x = 1.0;
    return (uint32_t)floor(x * 255.0 + 0.5);   /* x * 255 and + 0.5 are exact in FP64 */
}

/* Mutation (Sec. 3.3): child = parent + sigma * z on every parameter, with one
 * rounding of fma(sigma, z, parent) in FP64 and one rounding to FP32. */
static void mutate(const orc_world* w, const float* parent, uint32_t parent_slot, uint32_t step, float* child) {
    double z[4];
    double sigma = (double)w->d.mutation_sigma;
    for (uint64_t p = 0; p < w->P; ++p) {
        if (p % 4 == 0) {
            uint32_t ctr[4] = {parent_slot, step, ST_MUTATE, (uint32_t)(p / 4)};
            orc_gauss4(ctr, w->key, z);
        }
        child[p] = (float)fma(sigma, z[p % 4], (double)parent[p]);
    }
}

/* Storage copy of a master vector, dequantised exactly into doubles. */
static void quantize(const orc_world* w, const float* master, double* out) {
    if (w->d.wdtype == ORC_FP32) {
        for (uint64_t p = 0; p < w->P; ++p) out[p] = (double)master[p];
        return;
    }
    if (w->d.wdtype == ORC_BF16) {           /* weights and biases in BF16 */
        for (uint64_t p = 0; p < w->P; ++p) out[p] = bf16_value(orc_bf16_rne(master[p]));
        return;
    }
    /* FP8: per output row, scale = amax/448 (1 if the row is zero); q = RNE(w/scale)
     * saturated; value = q * scale.  Biases stay FP32. */
    layer_geom L[3];
    layers(w, L);
    for (int l = 0; l < 3; ++l) {
        for (uint32_t r = 0; r < L[l].rows; ++r) {
            const float* row = master + L[l].w_off + (uint64_t)r * L[l].cols;
            float amax = 0.0f;
            for (uint32_t c = 0; c < L[l].cols; ++c) {
                float a = fabsf(row[c]);
                if (a > amax) amax = a;
            }
            float scale = (amax > 0.0f) ? amax / 448.0f : 1.0f;
            for (uint32_t c = 0; c < L[l].cols; ++c) {
                uint8_t q = orc_fp8e4m3_rne_sat(row[c] / scale);
                out[L[l].w_off + (uint64_t)r * L[l].cols + c] = orc_fp8e4m3_decode(q) * (double)scale;
            }
            out[L[l].b_off + r] = (double)master[L[l].b_off + r];
        }
    }
    if (w->d.flags & ORC_EVOLVE_TEMPERATURE) out[w->P - 1] = (double)master[w->P - 1];   /* like a bias */
}

static double sqnorm(const float* v, uint64_t n) {
    double s = 0.0;
    for (uint64_t i = 0; i < n; ++i) s += (double)v[i] * (double)v[i];
    return s;
}

static int64_t new_node(orc_world* w, int64_t parent, uint32_t parent_slot, uint32_t step, uint32_t root) {
    if (w->n_nodes == w->nodes_cap) {
        size_t nc = w->nodes_cap ? 2 * w->nodes_cap : 1024;
        lineage_node* nn = (lineage_node*)realloc(w->nodes, nc * sizeof(lineage_node));
        if (!nn) return -1;
        w->nodes = nn;
        w->nodes_cap = nc;
    }
    lineage_node* n = &w->nodes[w->n_nodes];
    n->parent = parent; n->parent_slot = parent_slot; n->step = step; n->root = root;
    return (int64_t)w->n_nodes++;
}

/* Rebuild the FP32 master of a lineage node: initial weights of the root slot,
 * then every ancestor's mutation in birth order. */
static void materialize_node(const orc_world* w, int64_t id, float* out) {
    const lineage_node* n = &w->nodes[id];
    if (n->parent < 0) { init_weights(w, n->root, out); return; }
    float* tmp = (float*)malloc(w->P * sizeof(float));
    materialize_node(w, n->parent, tmp);
    mutate(w, tmp, n->parent_slot, n->step, out);
    free(tmp);
}

/* Give slot s a freshly initialised genome (init and write_state). */
static int seed_slot(orc_world* w, uint32_t s) {
    int64_t id = new_node(w, -1, 0, 0, s);
    if (id < 0) return fail("out of memory");
    w->node[s] = id;
    if (w->d.flags & ORC_COLOUR_VISION) init_colour(w, s, w->colour + 3 * (uint64_t)s);
    if (!w->materialize) { w->trait[s] = NAN; return 0; }   /* lineage mode: no traits */
    float* m = w->master + (uint64_t)s * w->P;
    init_weights(w, s, m);
    w->trait[s] = sqnorm(m, w->P);
    if (w->stored) quantize(w, m, w->stored + (uint64_t)s * w->P);
    return 0;
}

static void compute_stats_tail(orc_world* w) {
    orc_stats* st = &w->stats;
    st->step = w->step;
    uint64_t pop = 0;
    int64_t esum = 0;
    double tsum = 0.0;
    for (uint32_t s = 0; s < w->cap; ++s)
        if (w->alive[s]) { ++pop; esum += w->energy[s]; tsum += w->trait[s]; }
    double mean = pop ? tsum / (double)pop : 0.0, var = 0.0;
    for (uint32_t s = 0; s < w->cap; ++s)
        if (w->alive[s]) { double dv = w->trait[s] - mean; var += dv * dv; }
    st->population = pop;
    st->energy_total = (double)esum;
    st->trait_mean = mean;
    st->trait_var = pop ? var / (double)pop : 0.0;
    uint64_t rsum = 0;
    for (uint32_t c = 0; c < w->cells; ++c) rsum += w->res[c];
    st->resource_total = rsum;
    st->water_total = st->biomass_total = st->hp_total = 0;
    if (w->eco) {
        uint64_t ws = 0, es = 0, bs = 0, hs = 0;
        for (uint32_t c = 0; c < w->cells; ++c) { ws += (uint64_t)w->cw[c]; es += (uint64_t)w->ce[c]; bs += (uint64_t)w->cb[c]; }
        for (uint32_t s2 = 0; s2 < w->cap; ++s2)
            if (w->alive[s2]) { ws += (uint64_t)w->water[s2]; bs += (uint64_t)w->biomass[s2]; hs += (uint64_t)w->hp[s2]; }
        st->resource_total = es;
        st->water_total = ws;
        st->biomass_total = bs;
        st->hp_total = hs;
    }
}

/* Terrain (Sec. 3.2 "Terrain"; the paper's maps are figures, not a rule): a
 * value-noise field.  Lattice values v(i, j) = Philox(i + j NX, 0, 9, 0).x0 >> 27
 * (0..31) on an NX x NY torus lattice, NX = max(1, W / terrain_scale); a cell
 * takes the bilinear blend of its four lattice corners, in exact integers with
 * floor division, so heights stay in 0..31. */
static int32_t terrain_height(const orc_world* w, uint32_t x, uint32_t y) {
    const uint64_t W = w->W, H = w->H, L = (uint64_t)w->d.eco.terrain_scale;
    const uint64_t NX = W / L > 0 ? W / L : 1, NY = H / L > 0 ? H / L : 1;
    const uint64_t ax = (uint64_t)x * NX, ay = (uint64_t)y * NY;
    const uint64_t i = ax / W, j = ay / H, fx = ax % W, fy = ay % H;
    const uint64_t i1 = (i + 1) % NX, j1 = (j + 1) % NY;
    uint64_t v[4];
    const uint64_t corner[4][2] = {{i, j}, {i1, j}, {i, j1}, {i1, j1}};
    for (int k = 0; k < 4; ++k)
        v[k] = draw_x0(w->key, (uint32_t)(corner[k][0] + corner[k][1] * NX), 0, ST_TERRAIN, 0) >> 27;
    const uint64_t num = v[0] * (W - fx) * (H - fy) + v[1] * fx * (H - fy) + v[2] * (W - fx) * fy + v[3] * fx * fy;
    return (int32_t)(num / (W * H));
}

/* Flow directions: each cell's lowest 4-neighbour if strictly lower than the
 * cell itself (the first of N, E, S, W among equals), else none (-1). */
static uint32_t step_cell(const orc_world* w, uint32_t cell, int facing, int sign);
static void set_flow(orc_world* w) {
    for (uint32_t c = 0; c < w->cells; ++c) {
        int best = -1;
        int32_t bh = w->rock[c];
        for (int dd = 0; dd < 4; ++dd) {
            uint32_t n = step_cell(w, c, dd, +1);
            if (w->rock[n] < bh) { bh = w->rock[n]; best = dd; }
        }
        w->flowdir[c] = (int8_t)best;
    }
}

int orc_read_terrain(const orc_world* w, int32_t* rock) {
    if (!(w->d.flags & ORC_TERRAIN)) return fail("the world has no terrain");
    memcpy(rock, w->rock, (size_t)w->cells * 4);
    return 0;
}

int orc_write_terrain(orc_world* w, const int32_t* rock) {
    if (!(w->d.flags & ORC_TERRAIN)) return fail("the world has no terrain");
    for (uint32_t c = 0; c < w->cells; ++c)
        if (rock[c] < 0 || rock[c] > 31) return fail("heights must lie in 0..31");
    memcpy(w->rock, rock, (size_t)w->cells * 4);
    set_flow(w);
    return 0;
}

static int validate(const orc_desc* d) {
    if (!d) return fail("null desc");
    if (d->width < 1 || d->height < 1) return fail("empty grid");
    if ((uint64_t)d->width * d->height > (1ull << 31)) return fail("grid too large");
    if (d->window < 1 || d->window % 2 == 0) return fail("window must be odd");
    if (d->window > d->width || d->window > d->height) return fail("window larger than the grid");
    if (d->n_scalars != 4 && d->n_scalars != 8 && !((d->flags & ORC_ECOLOGY) && d->n_scalars == 12))
        return fail("n_scalars must be 4 or 8 (8 or 12 in the ecology)");
    if (d->n_actions < 5 || d->n_actions > 9 || d->n_actions == 6) return fail("n_actions must be 5, 7, 8 or 9");
    if (d->attack_enabled > 1) return fail("attack_enabled must be 0 or 1");
    if (d->attack_enabled && d->n_actions != ((d->flags & ORC_ECOLOGY) ? 9u : 7u))
        return fail("attacks need the seven-action head (nine in the ecology)");
    if (d->flags & ~(uint32_t)(ORC_FRONT_VISION | ORC_EVOLVE_TEMPERATURE | ORC_COLOUR_VISION | ORC_ECOLOGY | ORC_TERRAIN))
        return fail("unknown flags");
    if (d->flags & ORC_ECOLOGY) {
        const orc_ecology* e = &d->eco;
        if (d->n_actions != (d->attack_enabled ? 9u : 8u)) return fail("the ecology has eight actions (nine with attack)");
        if (e->attack_damage < 0 || e->attack_damage > (1 << 20)) return fail("attack_damage outside [0, 2^20]");
        if ((d->flags & ORC_TERRAIN) && (e->terrain_scale < 1 || e->sea_level < 0 || e->sea_level > 32 ||
                                         e->water_per_depth < 0))
            return fail("bad terrain parameters");
        if (d->n_scalars != 8 && d->n_scalars != 12) return fail("the ecology has 8 or 12 scalars");
        if (e->hp_max <= 0 || e->hp_child <= 0 || e->hp_child > e->hp_max) return fail("bad health limits");
        if (e->age_shift < 0 || e->age_shift > 31) return fail("age_shift outside [0, 31]");
        if (e->cap_water < 0 || e->cap_energy < 0 || e->cap_biomass < 0 || e->eat_water < 0 || e->eat_biomass < 0 ||
            e->w_cost < 0 || e->e_cost_move < 0 || e->hp_overspend < 0 || e->hp_heal < 0 || e->heal_energy < 0 ||
            e->w_init < 0 || e->b_init < 0 || e->w_child < 0 || e->b_child < 0 || e->b_repro < e->b_child ||
            e->water_site < 0 || e->energy_site < 0 || e->biomass_site < 0 || e->cell_energy_max < 0 || d->e_eat < 0 ||
            d->e_cost < 0 || d->e_child < 0)
            return fail("negative ecology amount");
        if (!(e->photo_rate >= 0.0f) || !(e->water_density >= 0.0f && e->water_density <= 1.0f) ||
            !(e->energy_density >= 0.0f && e->energy_density <= 1.0f) ||
            !(e->biomass_density >= 0.0f && e->biomass_density <= 1.0f))
            return fail("bad ecology rate or density");
    } else if (d->n_actions >= 8) {
        return fail("eight or nine actions need the ecology");
    }
    if ((d->flags & ORC_TERRAIN) && !(d->flags & ORC_ECOLOGY)) return fail("terrain needs the ecology");
    if (d->hidden1 < 1 || d->hidden2 < 1) return fail("hidden sizes must be positive");
    if (d->capacity < d->n_agents_init) return fail("capacity below the initial population");
    if ((uint64_t)d->n_agents_init > (uint64_t)d->width * d->height) return fail("more agents than cells");
    if (d->e_repro <= 0) return fail("e_repro must be positive");
    if (d->wdtype > ORC_FP8) return fail("unknown weight format");
    if (!(d->mutation_sigma >= 0.0f)) return fail("negative sigma");
    if (!(d->resource_density >= 0.0f && d->resource_density <= 1.0f)) return fail("density outside [0,1]");
    if (!(d->regrow_prob >= 0.0f && d->regrow_prob <= 1.0f)) return fail("regrow outside [0,1]");
    return 0;
}

typedef struct { uint32_t key, cell; } cell_key;
static int cmp_cell_key(const void* a, const void* b) {
    const cell_key* x = (const cell_key*)a;
    const cell_key* y = (const cell_key*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->cell < y->cell ? -1 : (x->cell > y->cell);
}

void orc_destroy(orc_world* w) {
    if (!w) return;
    free(w->pos); free(w->energy); free(w->age); free(w->facing); free(w->alive); free(w->action);
    free(w->uid); free(w->puid); free(w->occ); free(w->res); free(w->wall);
    free(w->master); free(w->stored); free(w->node); free(w->nodes); free(w->trait); free(w->colour);
    free(w->water); free(w->biomass); free(w->hp); free(w->cw); free(w->ce); free(w->cb);
    free(w->rock); free(w->flowdir);
    free(w);
}

orc_world* orc_create(const orc_desc* d, int materialize) {
    if (validate(d)) return NULL;
    orc_world* w = (orc_world*)calloc(1, sizeof(orc_world));
    if (!w) { fail("out of memory"); return NULL; }
    w->d = *d;
    w->W = d->width; w->H = d->height; w->cells = d->width * d->height; w->cap = d->capacity;
    w->S = d->window; w->R = (d->window - 1) / 2; w->ns = d->n_scalars;
    w->D = orc_input_dim(d); w->H1 = d->hidden1; w->H2 = d->hidden2; w->A = d->n_actions;
    w->P = orc_param_count(d);
    w->key[0] = (uint32_t)(d->seed & 0xFFFFFFFFu);
    w->key[1] = (uint32_t)(d->seed >> 32);
    w->materialize = materialize;
    uint32_t cap = w->cap;
    w->pos = (int32_t*)calloc(cap ? cap : 1, 4);    w->energy = (int32_t*)calloc(cap ? cap : 1, 4);
    w->age = (int32_t*)calloc(cap ? cap : 1, 4);    w->facing = (uint8_t*)calloc(cap ? cap : 1, 1);
    w->alive = (uint8_t*)calloc(cap ? cap : 1, 1);  w->action = (uint8_t*)calloc(cap ? cap : 1, 1);
    w->uid = (uint64_t*)calloc(cap ? cap : 1, 8);   w->puid = (uint64_t*)calloc(cap ? cap : 1, 8);
    w->node = (int64_t*)calloc(cap ? cap : 1, 8);   w->trait = (double*)calloc(cap ? cap : 1, 8);
    w->occ = (int32_t*)malloc((size_t)w->cells * 4);
    w->res = (uint8_t*)calloc(w->cells, 1);
    w->wall = (uint8_t*)calloc(w->cells, 1);
    w->colour = (float*)calloc((size_t)(cap ? cap : 1) * 3, sizeof(float));
    w->eco = (d->flags & ORC_ECOLOGY) != 0;
    w->water = (int32_t*)calloc(cap ? cap : 1, 4);   w->biomass = (int32_t*)calloc(cap ? cap : 1, 4);
    w->hp = (int32_t*)calloc(cap ? cap : 1, 4);
    w->cw = (int32_t*)calloc(w->cells, 4); w->ce = (int32_t*)calloc(w->cells, 4); w->cb = (int32_t*)calloc(w->cells, 4);
    w->rock = (int32_t*)calloc(w->cells, 4); w->flowdir = (int8_t*)calloc(w->cells, 1);
    if (materialize) {
        w->master = (float*)calloc((size_t)cap * w->P + 1, sizeof(float));
        if (d->wdtype != ORC_FP32) w->stored = (double*)calloc((size_t)cap * w->P + 1, sizeof(double));
    }
    if (!w->pos || !w->energy || !w->age || !w->facing || !w->alive || !w->action || !w->uid ||
        !w->puid || !w->node || !w->trait || !w->occ || !w->res || !w->wall || !w->colour || !w->water ||
        !w->biomass || !w->hp || !w->cw || !w->ce || !w->cb || !w->rock || !w->flowdir ||
        (materialize && (!w->master || (d->wdtype != ORC_FP32 && !w->stored)))) {
        orc_destroy(w);
        fail("out of memory");
        return NULL;
    }
    for (uint32_t c = 0; c < w->cells; ++c) w->occ[c] = -1;

    /* Placement: the n_agents_init cells with the smallest (Philox key, cell)
     * pairs, slot j taking the j-th smallest. */
    cell_key* ck = (cell_key*)malloc((size_t)w->cells * sizeof(cell_key));
    if (!ck) { orc_destroy(w); fail("out of memory"); return NULL; }
    for (uint32_t c = 0; c < w->cells; ++c) { ck[c].key = draw_x0(w->key, c, 0, ST_CELLKEY, 0); ck[c].cell = c; }
    qsort(ck, w->cells, sizeof(cell_key), cmp_cell_key);
    uint64_t rho = bern_threshold(d->resource_density);
    if (!w->eco) {
        for (uint32_t c = 0; c < w->cells; ++c) w->res[c] = ((uint64_t)draw_x0(w->key, c, 0, ST_RESINIT, 0) < rho) ? 1 : 0;
    } else {
        /* Water, energy and biomass sites from outputs 1, 2, 3 of the same block
         * (the single resource layer stays empty). */
        const uint64_t tw = bern_threshold(d->eco.water_density), te = bern_threshold(d->eco.energy_density),
                       tb = bern_threshold(d->eco.biomass_density);
        for (uint32_t c = 0; c < w->cells; ++c) {
            uint32_t ctr[4] = {c, 0u, ST_RESINIT, 0u}, x[4];
            orc_philox4x32_10(ctr, w->key, x);
            w->cw[c] = ((uint64_t)x[1] < tw) ? d->eco.water_site : 0;
            w->ce[c] = ((uint64_t)x[2] < te) ? d->eco.energy_site : 0;
            w->cb[c] = ((uint64_t)x[3] < tb) ? d->eco.biomass_site : 0;
        }
        if (d->flags & ORC_TERRAIN) {   /* rock from the noise field; the sea instead of water sites */
            for (uint32_t c = 0; c < w->cells; ++c) w->rock[c] = terrain_height(w, c % w->W, c / w->W);
            for (uint32_t c = 0; c < w->cells; ++c)
                w->cw[c] = (w->rock[c] < d->eco.sea_level) ? (d->eco.sea_level - w->rock[c]) * d->eco.water_per_depth : 0;
            set_flow(w);
        }
    }
    for (uint32_t j = 0; j < d->n_agents_init; ++j) {
        uint32_t cell = ck[j].cell;
        w->alive[j] = 1;
        w->pos[j] = (int32_t)cell;
        w->occ[cell] = (int32_t)j;
        w->facing[j] = (uint8_t)(draw_x0(w->key, j, 0, ST_FACING, 0) >> 30);
        w->energy[j] = d->e_init;
        w->age[j] = 0;
        if (w->eco) { w->water[j] = d->eco.w_init; w->biomass[j] = d->eco.b_init; w->hp[j] = d->eco.hp_max; }
        w->uid[j] = j;
        w->puid[j] = UINT64_MAX;
        int64_t id = new_node(w, -1, 0, 0, j);
        if (id < 0) { free(ck); orc_destroy(w); fail("out of memory"); return NULL; }
        w->node[j] = id;
        w->trait[j] = NAN;
        if (d->flags & ORC_COLOUR_VISION) init_colour(w, j, w->colour + 3 * (uint64_t)j);
    }
    free(ck);
    /* Initial weights: independent per agent, so the loop runs in parallel. */
    if (materialize) {
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t j = 0; j < (int64_t)d->n_agents_init; ++j) {
            float* m = w->master + (uint64_t)j * w->P;
            init_weights(w, (uint32_t)j, m);
            w->trait[j] = sqnorm(m, w->P);
            if (w->stored) quantize(w, m, w->stored + (uint64_t)j * w->P);
        }
    }
    w->uid_next = d->n_agents_init;
    w->step = 0;
    memset(&w->stats, 0, sizeof w->stats);
    compute_stats_tail(w);
    return w;
}

/* ------------------------------------------------------------------------- */
/* Observation and policy                                                    */
/* ------------------------------------------------------------------------- */
/* Colour vision (Sec. 3.2 "Sensors": a top-down rendered patch of three colour
 * channels and the local elevation difference).  A cell is drawn in its
 * occupant's colour; an empty cell holding a resource unit in green, a wall in
 * grey, anything else black; each channel as its 8-bit value times 2^-8.  The
 * torus is flat, so the elevation-difference channel is zero. */
static uint32_t sat255(int64_t v) { return v < 0 ? 0u : (v > 255 ? 255u : (uint32_t)v); }

static void render_cell(const orc_world* w, uint32_t cell, uint32_t own, double* v) {
    uint32_t q[3] = {0u, 0u, 0u};
    int32_t o = w->occ[cell];
    if (o >= 0) {
        for (int k = 0; k < 3; ++k) q[k] = orc_colour_byte(w->colour[3 * (uint64_t)o + k]);
    } else if (w->eco) {
        /* the ecology's cells: wall grey, else energy in red, biomass in green,
         * water in blue, each saturating at 255 */
        if (w->wall[cell]) {
            q[0] = q[1] = q[2] = 128u;
        } else {
            q[0] = sat255((int64_t)w->ce[cell] * 16);
            q[1] = sat255((int64_t)w->cb[cell] * 64);
            q[2] = sat255((int64_t)w->cw[cell] * 16);
        }
    } else if (w->res[cell]) {
        q[1] = 255u;
    } else if (w->wall[cell]) {
        q[0] = q[1] = q[2] = 128u;
    }
    for (int k = 0; k < 3; ++k) v[k] = ldexp((double)q[k], -8);
    /* the local difference in elevation: zero on the flat torus */
    v[3] = (w->d.flags & ORC_TERRAIN) ? ldexp((double)(w->rock[cell] - w->rock[own]), -3) : 0.0;
}

int orc_observe(const orc_world* w, uint32_t slot, double* x) {
    if (slot >= w->cap || !w->alive[slot]) return fail("slot not alive");
    int f = w->facing[slot];
    int64_t ax = w->pos[slot] % w->W, ay = w->pos[slot] / w->W;
    int dx = DX[f], dy = DY[f];
    int rx = -dy, ry = dx;                     /* the agent's right-hand direction */
    int S = (int)w->S, R = (int)w->R;
    /* Row 0 is the far front.  "Around": the agent's row is the middle one;
     * "Front": the agent's row is the last, so nothing behind it is seen. */
    int ahead0 = (w->d.flags & ORC_FRONT_VISION) ? S - 1 : R;
    for (int r = 0; r < S; ++r) {
        for (int c = 0; c < S; ++c) {
            int fwd = ahead0 - r, right = c - R;
            uint32_t cell = wrap_cell(w, ax + fwd * dx + right * rx, ay + fwd * dy + right * ry);
            int32_t o = w->occ[cell];
            double* v = x + 4 * (r * S + c);
            if (w->d.flags & ORC_COLOUR_VISION) { render_cell(w, cell, (uint32_t)w->pos[slot], v); continue; }
            if (w->eco) {   /* agent present, then water, energy, biomass levels (capped at 255) / 16 */
                v[0] = (o >= 0) ? 1.0 : 0.0;
                v[1] = ldexp((double)(w->cw[cell] < 255 ? w->cw[cell] : 255), -4);
                v[2] = ldexp((double)(w->ce[cell] < 255 ? w->ce[cell] : 255), -4);
                v[3] = ldexp((double)(w->cb[cell] < 255 ? w->cb[cell] : 255), -4);
                continue;
            }
            v[0] = (o >= 0) ? 1.0 : 0.0;
            v[1] = (double)w->res[cell];
            v[2] = (double)w->wall[cell];
            if (o >= 0) {
                int64_t eb = (int64_t)w->energy[o] * 8 / w->d.e_repro;
                if (eb < 0) eb = 0;
                if (eb > 7) eb = 7;
                v[3] = (double)eb;
            } else {
                v[3] = 0.0;
            }
        }
    }
    /* Scalars: internal (energy, age), external (resource here), eligibility,
     * then the 4-way compass when n_s = 8 (Sec. 3.2 "Sensors"). */
    double* s = x + 4 * S * S;
    int32_t E = w->energy[slot];
    int32_t age = w->age[slot] < 1024 ? w->age[slot] : 1024;
    if (w->eco) {
        /* internal: energy, age, water, biomass, health; external: the own cell's
         * water, energy, biomass levels; then the compass when n_s = 12. */
        uint32_t here = (uint32_t)w->pos[slot];
        s[0] = ldexp((double)E, -8);
        s[1] = ldexp((double)age, -10);
        s[2] = ldexp((double)w->water[slot], -8);
        s[3] = ldexp((double)w->biomass[slot], -3);
        s[4] = ldexp((double)w->hp[slot], -7);
        s[5] = ldexp((double)(w->cw[here] < 255 ? w->cw[here] : 255), -4);
        s[6] = ldexp((double)(w->ce[here] < 255 ? w->ce[here] : 255), -4);
        s[7] = ldexp((double)(w->cb[here] < 255 ? w->cb[here] : 255), -4);
        if (w->ns == 12)
            for (int k = 0; k < 4; ++k) s[8 + k] = (k == f) ? 1.0 : 0.0;
        return 0;
    }
    s[0] = ldexp((double)E, -8);
    s[1] = ldexp((double)age, -10);
    s[2] = (double)w->res[w->pos[slot]];
    s[3] = (E >= w->d.e_repro) ? 1.0 : 0.0;
    if (w->ns == 8)
        for (int k = 0; k < 4; ++k) s[4 + k] = (k == f) ? 1.0 : 0.0;
    return 0;
}

/* FP64 forward: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), l = W3 h2 + b3. */
static void forward(const orc_world* w, const double* theta, const double* x, double* logits) {
    layer_geom L[3];
    layers(w, L);
    double* h1 = (double*)malloc(sizeof(double) * (w->H1 + w->H2));
    double* h2 = h1 + w->H1;
    for (uint32_t j = 0; j < w->H1; ++j) {
        double acc = theta[L[0].b_off + j];
        for (uint32_t k = 0; k < w->D; ++k) acc += theta[L[0].w_off + (uint64_t)j * w->D + k] * x[k];
        h1[j] = acc > 0.0 ? acc : 0.0;
    }
    for (uint32_t i = 0; i < w->H2; ++i) {
        double acc = theta[L[1].b_off + i];
        for (uint32_t j = 0; j < w->H1; ++j) acc += theta[L[1].w_off + (uint64_t)i * w->H1 + j] * h1[j];
        h2[i] = acc > 0.0 ? acc : 0.0;
    }
    for (uint32_t a = 0; a < w->A; ++a) {
        double acc = theta[L[2].b_off + a];
        for (uint32_t i = 0; i < w->H2; ++i) acc += theta[L[2].w_off + (uint64_t)a * w->H2 + i] * h2[i];
        logits[a] = acc;
    }
    free(h1);
}

/* Softmax inverse CDF: m = max l, w_k = exp(l_k - m), C_k = w_0 + ... + w_k,
 * t = u C_{A-1}; the least k with t < C_k, else the last k with w_k > 0. */
/* Softmax with temperature tau = exp(log_tau) (Sec. 3.3): weights
 * exp((l_k - max l) / tau), the largest logits weighing exactly 1. */
int orc_sample_tempered(const double* l, int A, double log_tau, double u) {
    if (A < 1 || A > 9) return -1;
    double m = l[0];
    for (int k = 1; k < A; ++k) if (l[k] > m) m = l[k];
    const double inv_tau = exp(-log_tau);
    double wk[9], C[9], acc = 0.0;
    for (int k = 0; k < A; ++k) {
        wk[k] = (l[k] == m) ? 1.0 : exp((l[k] - m) * inv_tau);
        acc += wk[k];
        C[k] = acc;
    }
    double t = u * C[A - 1];
    for (int k = 0; k < A; ++k) if (t < C[k]) return k;
    for (int k = A - 1; k >= 0; --k) if (wk[k] > 0.0) return k;
    return A - 1;
}

int orc_sample(const double* l, int A, double u) { return orc_sample_tempered(l, A, 0.0, u); }

/* Weights of live slot s in logical order: storage (which=0) or master (which=1). */
static int slot_theta(orc_world* w, uint32_t s, int which, double* out) {
    if (s >= w->cap || !w->alive[s]) return fail("slot not alive");
    if (w->materialize) {
        const float* m = w->master + (uint64_t)s * w->P;
        if (which == 1 || w->d.wdtype == ORC_FP32) {
            for (uint64_t p = 0; p < w->P; ++p) out[p] = (double)m[p];
        } else {
            memcpy(out, w->stored + (uint64_t)s * w->P, w->P * sizeof(double));
        }
        return 0;
    }
    float* m = (float*)malloc(w->P * sizeof(float));
    if (!m) return fail("out of memory");
    materialize_node(w, w->node[s], m);
    if (which == 1) for (uint64_t p = 0; p < w->P; ++p) out[p] = (double)m[p];
    else quantize(w, m, out);
    free(m);
    return 0;
}

int orc_read_weights(orc_world* w, uint32_t slot, int which, double* out) {
    return slot_theta(w, slot, which, out);
}

int orc_agent_logits(orc_world* w, uint32_t slot, double* out) {
    if (slot >= w->cap || !w->alive[slot]) return fail("slot not alive");
    double* theta = (double*)malloc(w->P * sizeof(double));
    double* x = (double*)malloc(w->D * sizeof(double));
    if (!theta || !x) { free(theta); free(x); return fail("out of memory"); }
    int rc = slot_theta(w, slot, 0, theta);
    if (!rc) rc = orc_observe(w, slot, x);
    if (!rc) forward(w, theta, x, out);
    free(theta);
    free(x);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* The step                                                                  */
/* ------------------------------------------------------------------------- */
static int32_t min3(int32_t a, int32_t b, int32_t c) { int32_t m = a < b ? a : b; return m < c ? m : c; }

/* One live agent's resources and health after the moves (ecology).  It touches
 * only the cell it stands on, so the agents' order does not matter.
 *   eat: the chosen resource moves from the cell to the stomach, up to the eat
 *        amount, what the cell holds and the room left under the cap;
 *   costs: energy (rest the least) is destroyed; water is spent and returns to
 *        the cell; a resource that runs short is overspent (energy clamps at 0);
 *   damage: each overspent resource costs hp_overspend health, age costs
 *        age >> age_shift (small, growing with age), and each attack that
 *        struck the agent's cell this step costs attack_damage;
 *   death at health <= 0: water, energy and biomass carried go to the cell
 *        (a struck agent that dies counts as killed);
 *   otherwise healing: below full health, heal_energy energy buys hp_heal health
 *        (capped at hp_max); the agent ages. */
static void ecology_agent(orc_world* w, uint32_t s, uint32_t hits, orc_stats* st) {
    const orc_ecology* e = &w->d.eco;
    const uint32_t cell = (uint32_t)w->pos[s];
    const int a = w->action[s];
    int32_t E = w->energy[s], Wt = w->water[s], B = w->biomass[s], hp = w->hp[s];
    int32_t t = 0;
    if (a == ORC_EAT_ENERGY) {
        t = min3(w->d.e_eat, w->ce[cell], e->cap_energy - E);
        if (t > 0) { w->ce[cell] -= t; E += t; }
    } else if (a == ORC_EAT_WATER) {
        t = min3(e->eat_water, w->cw[cell], e->cap_water - Wt);
        if (t > 0) { w->cw[cell] -= t; Wt += t; }
    } else if (a == ORC_EAT_BIOMASS) {
        t = min3(e->eat_biomass, w->cb[cell], e->cap_biomass - B);
        if (t > 0) { w->cb[cell] -= t; B += t; }
    }
    if (t > 0) st->eaten++;
    int over = 0;
    E -= (a == ORC_REST) ? w->d.e_cost : e->e_cost_move;
    if (E < 0) { E = 0; over++; }
    int32_t spend = Wt < e->w_cost ? Wt : e->w_cost;
    Wt -= spend;
    w->cw[cell] += spend;
    if (spend < e->w_cost) over++;
    int64_t damage = (int64_t)over * e->hp_overspend + (w->age[s] >> e->age_shift) + (int64_t)hits * e->attack_damage;
    if ((int64_t)hp - damage <= 0) {
        w->cw[cell] += Wt; w->ce[cell] += E; w->cb[cell] += B;
        w->energy[s] = 0; w->water[s] = 0; w->biomass[s] = 0; w->hp[s] = 0;
        w->alive[s] = 0;
        w->occ[cell] = -1;
        st->deaths++;
        if (hits > 0) st->killed++;
        return;
    }
    hp -= (int32_t)damage;
    if (hp < e->hp_max && E >= e->heal_energy) {
        hp = (hp + e->hp_heal < e->hp_max) ? hp + e->hp_heal : e->hp_max;
        E -= e->heal_energy;
    }
    w->energy[s] = E; w->water[s] = Wt; w->biomass[s] = B; w->hp[s] = hp;
    w->age[s] += 1;
}

int orc_step(orc_world* w, const uint8_t* actions, double* logits_out, uint8_t* sampled_out) {
    const uint32_t cap = w->cap, A = w->A;
    const uint32_t step32 = (uint32_t)w->step;
    if (!actions && !w->materialize) return fail("sampling needs materialized weights");
    if (sampled_out && !w->materialize) return fail("sampling needs materialized weights");
    if (actions)
        for (uint32_t s = 0; s < cap; ++s)
            if (w->alive[s] && actions[s] >= A) return fail("action out of range");

    orc_stats* st = &w->stats;
    memset(st, 0, sizeof *st);

    /* 1. Live agents at the start of the step, ascending slot order. */
    uint8_t* live = (uint8_t*)malloc(cap ? cap : 1);
    memcpy(live, w->alive, cap);

    /* 2. Every live agent observes the pre-step state and picks an action. */
    if (logits_out) for (uint64_t i = 0; i < (uint64_t)cap * A; ++i) logits_out[i] = NAN;
    if (sampled_out) memset(sampled_out, 255, cap);
    if (w->materialize) {
#pragma omp parallel
        {
            double* x = (double*)malloc(w->D * sizeof(double));
            double* theta = (double*)malloc(w->P * sizeof(double));
            double l[9];
#pragma omp for schedule(dynamic, 16)
            for (int64_t si = 0; si < (int64_t)cap; ++si) {
                uint32_t s = (uint32_t)si;
                if (!live[s]) continue;
                slot_theta(w, s, 0, theta);
                orc_observe(w, s, x);
                forward(w, theta, x, l);
                uint32_t x0 = draw_x0(w->key, s, step32, ST_ACTION, 0);
                double u = (double)(x0 >> 8) * 0x1p-24;
                int a = (w->d.flags & ORC_EVOLVE_TEMPERATURE) ? orc_sample_tempered(l, (int)A, theta[w->P - 1], u)
                                                              : orc_sample(l, (int)A, u);
                if (logits_out) for (uint32_t k = 0; k < A; ++k) logits_out[(uint64_t)s * A + k] = l[k];
                if (sampled_out) sampled_out[s] = (uint8_t)a;
                w->action[s] = (uint8_t)a;
            }
            free(x);
            free(theta);
        }
    }
    for (uint32_t s = 0; s < cap; ++s) {
        if (!live[s]) continue;
        if (actions) w->action[s] = actions[s];
        st->action_hist[w->action[s]]++;
    }

    /* 3. Turns; then every FORWARD mover claims its target if the target was
     *    empty at the start of the step and is not a wall.  Lowest slot wins. */
    uint32_t* claim = (uint32_t*)malloc((size_t)w->cells * sizeof(uint32_t));
    int64_t* tgt = (int64_t*)malloc((size_t)(cap ? cap : 1) * sizeof(int64_t));
    for (uint32_t c = 0; c < w->cells; ++c) claim[c] = UINT32_MAX;
    for (uint32_t s = 0; s < cap; ++s) {
        if (!live[s]) continue;
        if (w->action[s] == ORC_TURN_L) w->facing[s] = (uint8_t)((w->facing[s] + 3) % 4);
        if (w->action[s] == ORC_TURN_R) w->facing[s] = (uint8_t)((w->facing[s] + 1) % 4);
    }
    for (uint32_t s = 0; s < cap; ++s) {
        tgt[s] = -1;
        if (!live[s] || w->action[s] != ORC_FORWARD) continue;
        uint32_t t = step_cell(w, (uint32_t)w->pos[s], w->facing[s], +1);
        if (w->occ[t] == -1 && !w->wall[t]) {
            tgt[s] = t;
            if (s < claim[t]) claim[t] = s;
        }
    }
    /* 4. Winners move; everyone else stays (no chains: targets were empty). */
    for (uint32_t s = 0; s < cap; ++s) {
        if (!live[s] || w->action[s] != ORC_FORWARD) continue;
        if (tgt[s] >= 0 && claim[tgt[s]] == s) {
            w->occ[w->pos[s]] = -1;
            w->occ[tgt[s]] = (int32_t)s;
            w->pos[s] = (int32_t)tgt[s];
            st->moves_ok++;
        } else {
            st->moves_blocked++;
        }
    }

    /* 4b. Attacks, after every move.  An attacker (which neither turned nor
     *     moved this step) strikes the cells 1, 2 and 3 ahead of it and one to
     *     either side of those: the 3x3 square directly in front.  On a torus
     *     smaller than the square it may wrap onto the attacker's own cell,
     *     which is never struck by its own attack.  All attacks land at once:
     *     an attacker standing in another attacker's square is killed too, and
     *     its own attack still lands.  Full strength: every struck agent dies.
     *     Ecology: the strikes on each cell are counted and cost health (5);
     *     an attacker strikes each distinct cell of its square once (on a torus
     *     narrower than three cells the square lists some cell twice). */
    uint32_t* struck = (uint32_t*)calloc(w->cells ? w->cells : 1, sizeof(uint32_t));
    if (w->d.attack_enabled) {
        const int attack = w->eco ? ORC_ATTACK_ECO : ORC_ATTACK;
        for (uint32_t s = 0; s < cap; ++s) {
            if (!live[s] || w->action[s] != attack) continue;
            const int f = w->facing[s], r = (f + 1) % 4;   /* the heading to the attacker's right */
            const int64_t x = w->pos[s] % (int32_t)w->W, y = w->pos[s] / (int32_t)w->W;
            uint32_t seen[9];
            int n_seen = 0;
            for (int ahead = 1; ahead <= 3; ++ahead)
                for (int side = -1; side <= 1; ++side) {
                    uint32_t c = wrap_cell(w, x + ahead * DX[f] + side * DX[r], y + ahead * DY[f] + side * DY[r]);
                    int dup = c == (uint32_t)w->pos[s];
                    for (int k = 0; k < n_seen; ++k) dup |= seen[k] == c;
                    if (dup) continue;
                    seen[n_seen++] = c;
                    struck[c] += 1;
                }
        }
    }

    /* 5. Ecology: every agent updates its resources and health (with the
     *    strikes on its cell).  Otherwise struck agents die where they stand and
     *    their carried energy returns to the cell as one resource unit (the
     *    resource layer holds 0 or 1 unit per cell); the others eat, pay the
     *    step cost and die at energy <= 0 (they carry nothing then); survivors
     *    age. */
    for (uint32_t s = 0; s < cap; ++s) {
        if (!live[s]) continue;
        uint32_t cell = (uint32_t)w->pos[s];
        if (w->eco) { ecology_agent(w, s, struck[cell], st); continue; }
        if (struck[cell]) {
            w->alive[s] = 0;
            w->occ[cell] = -1;
            w->res[cell] = 1;
            w->energy[s] = 0;
            st->deaths++;
            st->killed++;
            continue;
        }
        if (w->action[s] == ORC_EAT && w->res[cell] > 0) {
            w->res[cell] -= 1;
            w->energy[s] += w->d.e_eat;
            st->eaten++;
        }
        w->energy[s] -= w->d.e_cost;
        if (w->energy[s] <= 0) {
            w->alive[s] = 0;
            w->occ[cell] = -1;
            st->deaths++;
        } else {
            w->age[s] += 1;
        }
    }

    /* 6. Births.  Eligible parents target the cell directly behind them; it must
     *    be empty now and not a wall; lowest slot wins.  Winners in slot order
     *    take the free slots in ascending order until they run out. */
    for (uint32_t c = 0; c < w->cells; ++c) claim[c] = UINT32_MAX;
    for (uint32_t s = 0; s < cap; ++s) {
        tgt[s] = -1;
        if (!w->alive[s]) continue;
        int eligible = w->energy[s] >= w->d.e_repro && (A == 5 || w->action[s] == ORC_REPRODUCE);
        if (w->eco)   /* spare biomass and enough water to give the child */
            eligible = w->action[s] == ORC_REPRODUCE_ECO && w->energy[s] >= w->d.e_repro &&
                       w->water[s] >= w->d.eco.w_child && w->biomass[s] >= w->d.eco.b_repro;
        if (!eligible) continue;
        uint32_t t = step_cell(w, (uint32_t)w->pos[s], w->facing[s], -1);
        if (w->occ[t] == -1 && !w->wall[t]) {
            tgt[s] = t;
            if (s < claim[t]) claim[t] = s;
        } else {
            st->births_blocked_cell++;
        }
    }
    uint32_t* winners = (uint32_t*)malloc((size_t)(cap ? cap : 1) * sizeof(uint32_t));
    uint32_t* freel = (uint32_t*)malloc((size_t)(cap ? cap : 1) * sizeof(uint32_t));
    uint32_t n_win = 0, n_free = 0;
    for (uint32_t s = 0; s < cap; ++s) {
        if (tgt[s] >= 0) {
            if (claim[tgt[s]] == s) winners[n_win++] = s;
            else st->births_blocked_cell++;
        }
        if (!w->alive[s]) freel[n_free++] = s;
    }
    uint64_t births = 0;
    for (uint32_t k = 0; k < n_win; ++k) {
        uint32_t p = winners[k];
        if (k >= n_free) { st->births_blocked_capacity++; continue; }
        uint32_t c = freel[k];
        uint32_t t = (uint32_t)tgt[p];
        w->energy[p] -= w->d.e_child;
        if (w->eco) {
            w->water[p] -= w->d.eco.w_child;
            w->biomass[p] -= w->d.eco.b_child;
            w->water[c] = w->d.eco.w_child;
            w->biomass[c] = w->d.eco.b_child;
            w->hp[c] = w->d.eco.hp_child;
        }
        w->alive[c] = 1;
        w->pos[c] = (int32_t)t;
        w->occ[t] = (int32_t)c;
        w->facing[c] = w->facing[p];
        w->energy[c] = w->d.e_child;
        w->age[c] = 0;
        w->uid[c] = w->uid_next + k;
        w->puid[c] = w->uid[p];
        w->node[c] = new_node(w, w->node[p], p, step32, 0);
        if (w->d.flags & ORC_COLOUR_VISION)
            mutate_colour(w, w->colour + 3 * (uint64_t)p, p, step32, w->colour + 3 * (uint64_t)c);
        if (w->materialize) {
            float* cm = w->master + (uint64_t)c * w->P;
            mutate(w, w->master + (uint64_t)p * w->P, p, step32, cm);
            w->trait[c] = sqnorm(cm, w->P);
            if (w->stored) quantize(w, cm, w->stored + (uint64_t)c * w->P);
        } else {
            w->trait[c] = NAN;                   /* lineage mode: weights rebuilt on demand */
        }
        births++;
    }
    st->births = births;
    w->uid_next += births;
    free(winners);
    free(freel);

    /* 7. Regrowth: an empty cell gets one unit with probability regrow_prob.
     *    Ecology: photosynthesis instead, one energy unit with probability
     *    min(1, photo_rate * biomass) on every cell holding biomass, up to
     *    cell_energy_max (photo_rate * biomass is exact in FP64).  The draw of
     *    cell c is draw_cell (four cells per Philox block). */
    if (!w->eco) {
        uint64_t thr = bern_threshold(w->d.regrow_prob);
        for (uint32_t c = 0; c < w->cells; ++c) {
            if (w->res[c] != 0) continue;
            if ((uint64_t)draw_cell(w->key, c, step32) < thr) { w->res[c] = 1; st->regrown++; }
        }
    } else {
        for (uint32_t c = 0; c < w->cells; ++c) {
            if (w->cb[c] <= 0 || w->ce[c] >= w->d.eco.cell_energy_max) continue;
            double p = (double)w->d.eco.photo_rate * (double)w->cb[c];
            uint64_t thr = p >= 1.0 ? (1ull << 32) : (uint64_t)floor(p * 4294967296.0);
            if ((uint64_t)draw_cell(w->key, c, step32) < thr) { w->ce[c] += 1; st->regrown++; }
        }
        /* 7b. Terrain: all water on a cell with a flow direction moves one cell
         *     downhill, every cell at once (water is conserved). */
        if (w->d.flags & ORC_TERRAIN) {
            int32_t* nw = (int32_t*)calloc(w->cells ? w->cells : 1, 4);
            for (uint32_t c = 0; c < w->cells; ++c) {
                if (w->flowdir[c] < 0) nw[c] += w->cw[c];
                else nw[step_cell(w, c, w->flowdir[c], +1)] += w->cw[c];
            }
            memcpy(w->cw, nw, (size_t)w->cells * 4);
            free(nw);
        }
    }

    /* 8. Advance the clock and record the step's statistics. */
    w->step += 1;
    compute_stats_tail(w);
    free(struck);
    free(claim);
    free(tgt);
    free(live);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* State access                                                              */
/* ------------------------------------------------------------------------- */
size_t orc_state_bytes(const orc_world* w) {
    size_t n = 32 + (size_t)w->cap * (8 + 8 + 4 + 4 + 4 + 1 + 1 + 1) + (size_t)w->cells * (4 + 1 + 1);
    if (w->eco) n += (size_t)w->cap * 12 + (size_t)w->cells * 12;
    return n;
}

int orc_read_state(const orc_world* w, void* buf, size_t bytes) {
    if (bytes < orc_state_bytes(w)) return fail("state buffer too small");
    uint8_t* b = (uint8_t*)buf;
    size_t cap = w->cap, cells = w->cells;
    uint32_t hdr32[4] = {w->W, w->H, w->cap, 0};
    memcpy(b, &w->step, 8); memcpy(b + 8, &w->uid_next, 8); memcpy(b + 16, hdr32, 16);
    b += 32;
    memcpy(b, w->uid, cap * 8); b += cap * 8;
    memcpy(b, w->puid, cap * 8); b += cap * 8;
    memcpy(b, w->pos, cap * 4); b += cap * 4;
    memcpy(b, w->energy, cap * 4); b += cap * 4;
    memcpy(b, w->age, cap * 4); b += cap * 4;
    memcpy(b, w->occ, cells * 4); b += cells * 4;
    memcpy(b, w->facing, cap); b += cap;
    memcpy(b, w->alive, cap); b += cap;
    memcpy(b, w->action, cap); b += cap;
    memcpy(b, w->res, cells); b += cells;
    memcpy(b, w->wall, cells); b += cells;
    if (w->eco) {
        memcpy(b, w->water, cap * 4); b += cap * 4;
        memcpy(b, w->biomass, cap * 4); b += cap * 4;
        memcpy(b, w->hp, cap * 4); b += cap * 4;
        memcpy(b, w->cw, cells * 4); b += cells * 4;
        memcpy(b, w->ce, cells * 4); b += cells * 4;
        memcpy(b, w->cb, cells * 4);
    }
    return 0;
}

int orc_write_state(orc_world* w, const void* buf, size_t bytes) {
    if (bytes < orc_state_bytes(w)) return fail("state buffer too small");
    const uint8_t* b = (const uint8_t*)buf;
    uint32_t hdr32[4];
    memcpy(hdr32, b + 16, 16);
    if (hdr32[0] != w->W || hdr32[1] != w->H || hdr32[2] != w->cap) return fail("state shape mismatch");
    size_t cap = w->cap, cells = w->cells;
    uint8_t* was_alive = (uint8_t*)malloc(cap ? cap : 1);
    memcpy(was_alive, w->alive, cap);
    memcpy(&w->step, b, 8); memcpy(&w->uid_next, b + 8, 8);
    b += 32;
    memcpy(w->uid, b, cap * 8); b += cap * 8;
    memcpy(w->puid, b, cap * 8); b += cap * 8;
    memcpy(w->pos, b, cap * 4); b += cap * 4;
    memcpy(w->energy, b, cap * 4); b += cap * 4;
    memcpy(w->age, b, cap * 4); b += cap * 4;
    memcpy(w->occ, b, cells * 4); b += cells * 4;
    memcpy(w->facing, b, cap); b += cap;
    memcpy(w->alive, b, cap); b += cap;
    memcpy(w->action, b, cap); b += cap;
    memcpy(w->res, b, cells); b += cells;
    memcpy(w->wall, b, cells); b += cells;
    if (w->eco) {
        memcpy(w->water, b, cap * 4); b += cap * 4;
        memcpy(w->biomass, b, cap * 4); b += cap * 4;
        memcpy(w->hp, b, cap * 4); b += cap * 4;
        memcpy(w->cw, b, cells * 4); b += cells * 4;
        memcpy(w->ce, b, cells * 4); b += cells * 4;
        memcpy(w->cb, b, cells * 4);
    }
    for (uint32_t s = 0; s < w->cap; ++s) {
        if (w->alive[s] && !was_alive[s] && seed_slot(w, s)) { free(was_alive); return -1; }
    }
    free(was_alive);
    compute_stats_tail(w);
    return 0;
}

int orc_stats_get(const orc_world* w, orc_stats* out) {
    *out = w->stats;
    return 0;
}

int orc_read_colour(const orc_world* w, uint32_t slot, float out[3]) {
    if (!(w->d.flags & ORC_COLOUR_VISION)) return fail("the world has no colour trait");
    if (slot >= w->cap || !w->alive[slot]) return fail("slot not alive");
    for (int k = 0; k < 3; ++k) out[k] = w->colour[3 * (uint64_t)slot + k];
    return 0;
}

int orc_write_colour(orc_world* w, uint32_t slot, const float in[3]) {
    if (!(w->d.flags & ORC_COLOUR_VISION)) return fail("the world has no colour trait");
    if (slot >= w->cap || !w->alive[slot]) return fail("slot not alive");
    for (int k = 0; k < 3; ++k) {
        if (!isfinite(in[k])) return fail("colour must be finite");
        w->colour[3 * (uint64_t)slot + k] = in[k];
    }
    return 0;
}
