/*
 * Seeded synthetic workload generator for the docking screen.
 *
 * This module only DRAWS inputs: protein "pocket" atoms, tree-shaped ligands
 * with 3D coordinates, rotatable-bond flags, atom types, the rigid-start
 * quaternion and translation sets.  It contains none of the docking
 * arithmetic (no potentials, no interpolation, no scoring, no search).
 * Both the GPU path and the CPU oracle consume what it produces.
 *
 * Randomness: every ligand owns an independent splitmix64 stream keyed by
 * (seed, stream, ligand id), so ligand g is identical whichever batch or
 * chunk it is generated in.  splitmix64 is Steele, Lea and Flood's
 * published generator (OOPSLA 2014): an additive Weyl sequence passed
 * through a 64-bit finaliser.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define GEN_MAX_ATOMS 128
#define GEN_MAX_DEG 4

static inline uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s; } rng_t;

static inline uint64_t rng_next(rng_t *r)
{
    r->s += 0x9E3779B97F4A7C15ULL;
    return sm_mix(r->s);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double rng_u01(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [0, m) (m small, so the modulo bias is < 2^-50) */
static inline int rng_int(rng_t *r, int m) { return (int)(rng_next(r) % (uint64_t)m); }

static inline double rng_normal(rng_t *r)
{
    /* Box-Muller; u1 in (0, 1] */
    double u1 = 1.0 - rng_u01(r);
    double u2 = rng_u01(r);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

static inline uint64_t key_of(uint64_t seed, uint64_t stream, uint64_t id)
{
    return sm_mix(sm_mix(sm_mix(seed) ^ (stream * 0xD6E8FEB86659FD93ULL)) + id);
}

/* Library distribution.  fixed_n > 0 / fixed_b >= 0 override the draws. */
typedef struct {
    double n_mean, n_sd;
    int32_t n_min, n_max;
    double tail_p;          /* probability of a heavy-tail ligand */
    int32_t tail_min, tail_max;
    double b_mean;          /* Poisson mean of the rotatable-bond count */
    int32_t b_min, b_max;
    int32_t fixed_n;        /* > 0: every ligand has exactly this many atoms */
    int32_t fixed_b;        /* >= 0: every ligand has exactly this many rotatable bonds */
    int32_t n_types;
    float offset_range;     /* input conformers are translated by U[-r, r]^3 */
} gen_lib_params;

static int draw_n(rng_t *r, const gen_lib_params *p)
{
    /* always consume the same number of draws so later draws do not depend on branches */
    double ut = rng_u01(r);
    double ui = rng_u01(r);
    double z = rng_normal(r);
    if (p->fixed_n > 0) return p->fixed_n;
    if (p->tail_p > 0.0 && ut < p->tail_p) {
        int span = p->tail_max - p->tail_min + 1;
        int v = p->tail_min + (int)(ui * span);
        return v > p->tail_max ? p->tail_max : v;
    }
    long v = lround(p->n_mean + p->n_sd * z);
    if (v < p->n_min) v = p->n_min;
    if (v > p->n_max) v = p->n_max;
    return (int)v;
}

static int draw_b(rng_t *r, const gen_lib_params *p)
{
    double u = rng_u01(r);
    if (p->fixed_b >= 0) return p->fixed_b;
    /* inverse CDF of Poisson(b_mean) */
    double pk = exp(-p->b_mean), cdf = pk;
    int k = 0;
    while (u > cdf && k < 1000) {
        k++;
        pk *= p->b_mean / k;
        cdf += pk;
    }
    if (k < p->b_min) k = p->b_min;
    if (k > p->b_max) k = p->b_max;
    return k;
}

/* Number of atoms of ligands [first_id, first_id + n_lig). */
int gen_ligand_sizes(uint64_t seed, uint64_t stream, int64_t first_id, int32_t n_lig,
                     const gen_lib_params *p, int32_t *n_atoms)
{
    for (int32_t l = 0; l < n_lig; ++l) {
        rng_t r = {key_of(seed, stream, (uint64_t)(first_id + l))};
        n_atoms[l] = draw_n(&r, p);
    }
    return 0;
}

#define BOND_LEN 1.5
#define MIN_NONBONDED 2.6
#define COS_MIN_ANGLE (-0.17364817766693033) /* cos(100 degrees) */

/* Grows one tree-shaped conformer; returns 0 on success, -1 when stuck. */
static int grow_tree(rng_t *r, int n, double pos[][3], int parent[], int deg[], int nbr[][GEN_MAX_DEG])
{
    pos[0][0] = pos[0][1] = pos[0][2] = 0.0;
    deg[0] = 0;
    parent[0] = -1;
    for (int i = 1; i < n; ++i) {
        int placed = 0;
        for (int tries = 0; tries < 400 && !placed; ++tries) {
            int par = rng_int(r, i);
            double z = 2.0 * rng_u01(r) - 1.0;
            double phi = 2.0 * M_PI * rng_u01(r);
            if (deg[par] >= GEN_MAX_DEG) continue;
            double s = sqrt(1.0 - z * z);
            double d[3] = {s * cos(phi), s * sin(phi), z};
            double c[3];
            for (int k = 0; k < 3; ++k) c[k] = pos[par][k] + BOND_LEN * d[k];
            int ok = 1;
            for (int q = 0; q < deg[par] && ok; ++q) {
                int nb = nbr[par][q];
                double v[3], vn = 0.0, dot = 0.0;
                for (int k = 0; k < 3; ++k) { v[k] = pos[nb][k] - pos[par][k]; vn += v[k] * v[k]; }
                vn = sqrt(vn);
                for (int k = 0; k < 3; ++k) dot += d[k] * v[k] / vn;
                if (dot > COS_MIN_ANGLE) ok = 0;
            }
            for (int j = 0; j < i && ok; ++j) {
                if (j == par) continue;
                int near = 0;
                for (int q = 0; q < deg[par]; ++q) near |= (nbr[par][q] == j);
                if (near) continue;
                double dd = 0.0;
                for (int k = 0; k < 3; ++k) { double t = c[k] - pos[j][k]; dd += t * t; }
                if (dd < MIN_NONBONDED * MIN_NONBONDED) ok = 0;
            }
            if (!ok) continue;
            for (int k = 0; k < 3; ++k) pos[i][k] = c[k];
            parent[i] = par;
            deg[i] = 1;
            nbr[i][0] = par;
            nbr[par][deg[par]++] = i;
            placed = 1;
        }
        if (!placed) return -1;
    }
    return 0;
}

/*
 * Fills ligands [first_id, first_id + n_lig).  atom_off is the CSR offset
 * array (n_lig + 1) built from gen_ligand_sizes; ligand l has n_l - 1 bonds
 * stored from bond index atom_off[l] - l.  Per ligand: xyz (FP32, AoS),
 * types, bonds (local atom indices, pairs), rotatable flags.  n_rot_out
 * (may be NULL) receives each ligand's rotatable-bond count.
 * Returns the number of ligands that needed more than one growth attempt.
 */
int gen_ligands(uint64_t seed, uint64_t stream, int64_t first_id, int32_t n_lig,
                const gen_lib_params *p, const int32_t *atom_off,
                float *xyz, uint8_t *type, int32_t *bonds, uint8_t *rot, int32_t *n_rot_out)
{
    int restarts = 0;
    /* weights 1/(1+t) for the ligand type draw */
    double cdf[64];
    int T = p->n_types < 64 ? p->n_types : 64;
    double tot = 0.0;
    for (int t = 0; t < T; ++t) { tot += 1.0 / (1.0 + t); cdf[t] = tot; }

#pragma omp parallel for schedule(dynamic, 64) reduction(+ : restarts)
    for (int32_t l = 0; l < n_lig; ++l) {
        rng_t r = {key_of(seed, stream, (uint64_t)(first_id + l))};
        int n = draw_n(&r, p);
        int btarget = draw_b(&r, p);
        double pos[GEN_MAX_ATOMS][3];
        int parent[GEN_MAX_ATOMS], deg[GEN_MAX_ATOMS], nbr[GEN_MAX_ATOMS][GEN_MAX_DEG];
        int attempt = 0;
        while (grow_tree(&r, n, pos, parent, deg, nbr) != 0) {
            attempt++;
            if (attempt > 1000) break; /* never observed; output stays a valid tree below */
        }
        if (attempt) restarts++;

        /* random relabelling of atoms so parents need not precede children */
        int perm[GEN_MAX_ATOMS];
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int i = n - 1; i > 0; --i) {
            int j = rng_int(&r, i + 1);
            int t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
        double off[3];
        for (int k = 0; k < 3; ++k) off[k] = (2.0 * rng_u01(&r) - 1.0) * p->offset_range;
        int64_t a0 = atom_off[l];
        for (int i = 0; i < n; ++i) {
            int64_t dst = a0 + perm[i];
            for (int k = 0; k < 3; ++k) xyz[3 * dst + k] = (float)(pos[i][k] + off[k]);
            double u = rng_u01(&r) * tot;
            int t = 0;
            while (t < T - 1 && u >= cdf[t]) t++;
            type[dst] = (uint8_t)t;
        }
        /* bonds: child i (1..n-1) to its parent, endpoints in random order */
        int64_t b0 = atom_off[l] - l;
        int nonterm[GEN_MAX_ATOMS], n_nonterm = 0;
        for (int i = 1; i < n; ++i) {
            int u = perm[parent[i]], v = perm[i];
            if (rng_u01(&r) < 0.5) { int t = u; u = v; v = t; }
            bonds[2 * (b0 + i - 1)] = u;
            bonds[2 * (b0 + i - 1) + 1] = v;
            rot[b0 + i - 1] = 0;
            if (deg[i] >= 2 && deg[parent[i]] >= 2) nonterm[n_nonterm++] = i - 1;
        }
        int b = btarget < n_nonterm ? btarget : n_nonterm;
        for (int k = 0; k < b; ++k) { /* partial Fisher-Yates: b distinct non-terminal bonds */
            int j = k + rng_int(&r, n_nonterm - k);
            int t = nonterm[k]; nonterm[k] = nonterm[j]; nonterm[j] = t;
            rot[b0 + nonterm[k]] = 1;
        }
        if (n_rot_out) n_rot_out[l] = b;
    }
    return restarts;
}

/* Protein atoms uniform in the spherical shell r_in <= |x - center| <= r_out, types uniform. */
int gen_pocket_atoms(uint64_t seed, uint64_t stream, uint64_t pocket_id, int32_t n_prot, int32_t n_types,
                     const double center[3], double r_in, double r_out, float *xyz, int32_t *type)
{
    rng_t r = {key_of(seed, stream, pocket_id)};
    for (int32_t j = 0; j < n_prot; ++j) {
        double u = rng_u01(&r);
        double rad = cbrt(r_in * r_in * r_in + u * (r_out * r_out * r_out - r_in * r_in * r_in));
        double z = 2.0 * rng_u01(&r) - 1.0;
        double phi = 2.0 * M_PI * rng_u01(&r);
        double s = sqrt(1.0 - z * z);
        xyz[3 * j + 0] = (float)(center[0] + rad * s * cos(phi));
        xyz[3 * j + 1] = (float)(center[1] + rad * s * sin(phi));
        xyz[3 * j + 2] = (float)(center[2] + rad * z);
        type[j] = rng_int(&r, n_types);
    }
    return 0;
}

/* t_0 = center; t_1..T-1 = center + points uniform in a ball of the given radius. */
int gen_translations(uint64_t seed, uint64_t stream, int32_t n_trans, double radius, const double center[3],
                     float *out)
{
    rng_t r = {key_of(seed, stream, 0x7472616e73ULL)};
    for (int k = 0; k < 3; ++k) out[k] = (float)center[k];
    for (int32_t i = 1; i < n_trans; ++i) {
        double v[3], n2;
        do {
            for (int k = 0; k < 3; ++k) v[k] = 2.0 * rng_u01(&r) - 1.0;
            n2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        } while (n2 > 1.0);
        for (int k = 0; k < 3; ++k) out[3 * i + k] = (float)(center[k] + radius * v[k]);
    }
    return 0;
}

/*
 * Deterministic near-uniform rotation set: the super-Fibonacci spiral of
 * Alexa (CVPR 2022).  Output quaternions (w, x, y, z), rounded to FP32.
 */
int gen_quaternions(int32_t n, float *out)
{
    const double phi = sqrt(2.0);
    const double psi = 1.533751168755204288118041; /* real root of psi^4 = psi + 4 */
    for (int32_t i = 0; i < n; ++i) {
        double s = i + 0.5;
        double rr = sqrt(s / n), RR = sqrt(1.0 - s / n);
        double alpha = 2.0 * M_PI * s / phi, beta = 2.0 * M_PI * s / psi;
        double x = rr * sin(alpha), y = rr * cos(alpha), z = RR * sin(beta), w = RR * cos(beta);
        out[4 * i + 0] = (float)w;
        out[4 * i + 1] = (float)x;
        out[4 * i + 2] = (float)y;
        out[4 * i + 3] = (float)z;
    }
    return 0;
}
