/*
 * FP64 CPU oracle of the rigid-receptor docking screen.
 *
 * TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the CPU-baseline leg of
 * the benchmark call it; the product (HIP) path never does, and the two share
 * no code.  Every routine below is the plain definition of one step, written
 * for a reader to check against the method by eye: no blocking, no fusion, no
 * incremental scoring.  A pose is always rescored from scratch.
 *
 * The method (paper §2, "LIGATE CADD Workflow"): ligands are docked into a
 * rigid binding site by a geometric search with multiple restarts, each pose
 * is scored by a geometric function, and a ligand's score is the score of its
 * best pose; the library is then ranked.  Here the restarts are rigid
 * quaternion x translation starts, each followed by one greedy pass of
 * per-fragment torsion sweeps, and the score is a trilinear lookup into
 * precomputed per-atom-type receptor grids plus an intra-ligand clash term.
 *
 * Units: Angstrom and kcal/mol-like energies; lower scores are better.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_ATOMS 128
#define OR_MAX_TORS 16
#define OR_MAX_DEG 4
#define OR_MAX_PAIRS (OR_MAX_ATOMS * (OR_MAX_ATOMS - 1) / 2)

/* Per-ligand status codes, in the order the checks are made. */
enum {
    OR_LIG_OK = 0,
    OR_LIG_NATOMS = 1,       /* n < 1 or n > 128 */
    OR_LIG_TYPE = 2,         /* an atom type >= n_types */
    OR_LIG_NBONDS = 3,       /* bond count != n - 1 */
    OR_LIG_BOND_INDEX = 4,   /* bond endpoint outside [0, n) or a self bond */
    OR_LIG_DEGREE = 5,       /* an atom with more than 4 bonds */
    OR_LIG_NOT_TREE = 6,     /* the bond graph is not connected */
    OR_LIG_TERMINAL_ROT = 7, /* a rotatable bond with an endpoint of degree 1 */
    OR_LIG_NTORSIONS = 8     /* more than 16 rotatable bonds */
};

/* ------------------------------------------------------------------------------------------ */
/* Receptor grids                                                                              */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    int32_t nx, ny, nz, n_types;
    double origin[3]; /* node (i, j, k) sits at origin + spacing * (i, j, k) */
    double spacing;
    int32_t periodic; /* 0: clamp + quadratic restraint outside the box, 1: periodic wrap */
    double w_out;     /* restraint weight (clamp mode) */
} or_frame;

typedef struct {
    const double *R, *eps, *q; /* per atom type: radius, well depth, charge */
    double cap;                /* the summed grid value is capped at this */
    double r_min;              /* distances are floored at this */
    double coulomb_k;          /* Coulomb constant over the dielectric */
} or_potential;

/*
 * Pair energy between a probe of type a and a protein atom of type b at
 * distance r: a 6-12 Lennard-Jones-like well with minimum at r0 = R_a + R_b
 * and depth sqrt(eps_a eps_b), plus a Coulomb-like term; r is floored at r_min.
 */
double or_pair_energy(double r, int a, int b, const or_potential *pot)
{
    double rt = r > pot->r_min ? r : pot->r_min;
    double r0 = pot->R[a] + pot->R[b];
    double eps = sqrt(pot->eps[a] * pot->eps[b]);
    double s6 = pow(r0 / rt, 6.0);
    return eps * (s6 * s6 - 2.0 * s6) + pot->coulomb_k * pot->q[a] * pot->q[b] / rt;
}

/* Grid value of type t at node (i, j, k): the capped sum over all protein atoms. */
double or_grid_node(const or_frame *f, const or_potential *pot, const float *prot_xyz,
                    const int32_t *prot_type, int32_t n_prot, int t, int i, int j, int k)
{
    double node[3] = {f->origin[0] + f->spacing * i, f->origin[1] + f->spacing * j,
                      f->origin[2] + f->spacing * k};
    double sum = 0.0;
    for (int32_t p = 0; p < n_prot; ++p) {
        double dx = node[0] - (double)prot_xyz[3 * p + 0];
        double dy = node[1] - (double)prot_xyz[3 * p + 1];
        double dz = node[2] - (double)prot_xyz[3 * p + 2];
        sum += or_pair_energy(sqrt(dx * dx + dy * dy + dz * dz), t, prot_type[p], pot);
    }
    return sum < pot->cap ? sum : pot->cap;
}

/* All grids, [t][k][j][i] with i (x) fastest; stored in FP32 as the method stores them. */
int or_build_grids(const or_frame *f, const or_potential *pot, const float *prot_xyz, const int32_t *prot_type,
                   int32_t n_prot, float *out32, double *out64)
{
    int64_t nxy = (int64_t)f->nx * f->ny, nxyz = nxy * f->nz;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int t = 0; t < f->n_types; ++t)
        for (int k = 0; k < f->nz; ++k)
            for (int j = 0; j < f->ny; ++j)
                for (int i = 0; i < f->nx; ++i) {
                    double v = or_grid_node(f, pot, prot_xyz, prot_type, n_prot, t, i, j, k);
                    int64_t idx = t * nxyz + k * nxy + (int64_t)j * f->nx + i;
                    out32[idx] = (float)v;
                    if (out64) out64[idx] = v;
                }
    return 0;
}

/*
 * Trilinear interpolation of grid t at point x (FP64 arithmetic on the FP32 grid).
 * Clamp mode: the point is clamped into the box, the cell is the one holding the
 * clamped point (the last cell along an axis for points on its upper face), and a
 * restraint w_out * |x - clamp(x)|^2 is added, so the value is continuous everywhere.
 * Periodic mode: indices wrap modulo the grid size (used to test translation covariance).
 */
double or_lookup(const or_frame *f, const float *G, int t, const double x[3])
{
    int n[3] = {f->nx, f->ny, f->nz};
    int64_t i0[3], i1[3];
    double fr[3], restraint = 0.0;
    for (int d = 0; d < 3; ++d) {
        double u = (x[d] - f->origin[d]) / f->spacing;
        if (f->periodic) {
            double fl = floor(u);
            fr[d] = u - fl;
            int64_t m = ((int64_t)fl % n[d] + n[d]) % n[d];
            i0[d] = m;
            i1[d] = (m + 1) % n[d];
        } else {
            double uc = u < 0.0 ? 0.0 : (u > n[d] - 1 ? n[d] - 1 : u);
            double fl = floor(uc);
            if (fl > n[d] - 2) fl = n[d] - 2;
            i0[d] = (int64_t)fl;
            i1[d] = i0[d] + 1;
            fr[d] = uc - fl;
            double lo = f->origin[d], hi = f->origin[d] + f->spacing * (n[d] - 1);
            double xc = x[d] < lo ? lo : (x[d] > hi ? hi : x[d]);
            restraint += (x[d] - xc) * (x[d] - xc);
        }
    }
    /* The trilinear polynomial sum_c prod_d (c_d ? f_d : 1 - f_d) G[corner c], evaluated as
       linear interpolations along x, then y, then z, each as lo + f (hi - lo): the same
       polynomial, and exactly the common value on a cell whose eight corners are equal
       (e.g. all at the cap), so such poses tie exactly. */
    const float *g = G + (int64_t)t * n[0] * n[1] * n[2];
    double cyz[2][2];
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy) {
            int64_t kk = cz ? i1[2] : i0[2], jj = cy ? i1[1] : i0[1];
            double lo = g[(kk * n[1] + jj) * n[0] + i0[0]], hi = g[(kk * n[1] + jj) * n[0] + i1[0]];
            cyz[cz][cy] = lo + fr[0] * (hi - lo);
        }
    double cz0 = cyz[0][0] + fr[1] * (cyz[0][1] - cyz[0][0]);
    double cz1 = cyz[1][0] + fr[1] * (cyz[1][1] - cyz[1][0]);
    double v = cz0 + fr[2] * (cz1 - cz0);
    if (!f->periodic) v += f->w_out * restraint;
    return v;
}

/* ------------------------------------------------------------------------------------------ */
/* Rotations                                                                                   */
/* ------------------------------------------------------------------------------------------ */

/* Active rotation matrix of the normalised quaternion q = (w, x, y, z) (Hamilton convention). */
void or_quat_matrix(const double qin[4], double Rm[9])
{
    double nrm = sqrt(qin[0] * qin[0] + qin[1] * qin[1] + qin[2] * qin[2] + qin[3] * qin[3]);
    double w = qin[0] / nrm, x = qin[1] / nrm, y = qin[2] / nrm, z = qin[3] / nrm;
    Rm[0] = 1 - 2 * (y * y + z * z); Rm[1] = 2 * (x * y - w * z);     Rm[2] = 2 * (x * z + w * y);
    Rm[3] = 2 * (x * y + w * z);     Rm[4] = 1 - 2 * (x * x + z * z); Rm[5] = 2 * (y * z - w * x);
    Rm[6] = 2 * (x * z - w * y);     Rm[7] = 2 * (y * z + w * x);     Rm[8] = 1 - 2 * (x * x + y * y);
}

/* Rodrigues' formula: v rotated by angle th (right hand) about the unit axis u. */
void or_rodrigues(const double u[3], double th, const double v[3], double out[3])
{
    double c = cos(th), s = sin(th);
    double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    double ud = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
    for (int d = 0; d < 3; ++d) out[d] = v[d] * c + cr[d] * s + u[d] * ud * (1.0 - c);
}

/* ------------------------------------------------------------------------------------------ */
/* Ligand topology                                                                             */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    int n, status, B, n_pairs;
    double xref[OR_MAX_ATOMS][3]; /* input conformer minus its unweighted centroid */
    int type[OR_MAX_ATOMS];
    int tor_a[OR_MAX_TORS], tor_b[OR_MAX_TORS]; /* axis a -> b; a on the core side */
    int tor_bond[OR_MAX_TORS];                  /* index of the bond in the input list */
    unsigned char moving[OR_MAX_TORS][OR_MAX_ATOMS];
    unsigned char core[OR_MAX_ATOMS];
    int pair_i[OR_MAX_PAIRS], pair_j[OR_MAX_PAIRS]; /* clash pairs: tree distance >= 3 */
} or_lig;

typedef struct {
    const int32_t *atom_off;
    const float *xyz;
    const uint8_t *type;
    const int32_t *bond_off;
    const int32_t *bonds;
    const uint8_t *rot;
    int32_t n_types;
} or_library;

/* Atoms reachable from `start` without using the edge (block_u, block_v); mask out[n]. */
static void reach(int n, int deg[], int nbr[][OR_MAX_DEG], int start, int block_u, int block_v,
                  const unsigned char *cut_edge_ok /* NULL or per-atom-pair filter not used */,
                  unsigned char out[])
{
    (void)cut_edge_ok;
    int stack[OR_MAX_ATOMS], sp = 0;
    memset(out, 0, (size_t)n);
    out[start] = 1;
    stack[sp++] = start;
    while (sp) {
        int x = stack[--sp];
        for (int q = 0; q < deg[x]; ++q) {
            int y = nbr[x][q];
            if ((x == block_u && y == block_v) || (x == block_v && y == block_u)) continue;
            if (!out[y]) { out[y] = 1; stack[sp++] = y; }
        }
    }
}

/*
 * Validates ligand l and derives everything the search needs from its bond tree:
 * the reference conformer, the rigid fragments (components left after cutting the
 * rotatable bonds), the core (the largest fragment; ties go to the one holding the
 * lowest atom index), each torsion's axis a -> b with a on the core side and its
 * moving set (the atoms on b's side), the sweep order (larger moving sets first,
 * ties by input bond index, which runs from the core outwards) and the clash pairs
 * (atom pairs three or more bonds apart).
 */
int or_ligand(const or_library *lib, int64_t l, or_lig *L)
{
    int32_t a0 = lib->atom_off[l], n = lib->atom_off[l + 1] - a0;
    int32_t b0 = lib->bond_off[l], nb = lib->bond_off[l + 1] - b0;
    memset(L, 0, sizeof(*L));
    L->n = n;
    if (n < 1 || n > OR_MAX_ATOMS) { L->status = OR_LIG_NATOMS; return L->status; }
    for (int i = 0; i < n; ++i)
        if (lib->type[a0 + i] >= lib->n_types) { L->status = OR_LIG_TYPE; return L->status; }
    if (nb != n - 1) { L->status = OR_LIG_NBONDS; return L->status; }
    for (int e = 0; e < nb; ++e) {
        int u = lib->bonds[2 * (b0 + e)], v = lib->bonds[2 * (b0 + e) + 1];
        if (u < 0 || u >= n || v < 0 || v >= n || u == v) { L->status = OR_LIG_BOND_INDEX; return L->status; }
    }
    int deg[OR_MAX_ATOMS] = {0};
    for (int e = 0; e < nb; ++e) { deg[lib->bonds[2 * (b0 + e)]]++; deg[lib->bonds[2 * (b0 + e) + 1]]++; }
    for (int i = 0; i < n; ++i)
        if (deg[i] > OR_MAX_DEG) { L->status = OR_LIG_DEGREE; return L->status; }
    int nbr[OR_MAX_ATOMS][OR_MAX_DEG];
    int fill[OR_MAX_ATOMS] = {0};
    for (int e = 0; e < nb; ++e) {
        int u = lib->bonds[2 * (b0 + e)], v = lib->bonds[2 * (b0 + e) + 1];
        nbr[u][fill[u]++] = v;
        nbr[v][fill[v]++] = u;
    }
    unsigned char seen[OR_MAX_ATOMS];
    reach(n, deg, nbr, 0, -1, -1, NULL, seen);
    for (int i = 0; i < n; ++i)
        if (!seen[i]) { L->status = OR_LIG_NOT_TREE; return L->status; }
    int nrot = 0;
    for (int e = 0; e < nb; ++e) {
        if (!lib->rot[b0 + e]) continue;
        int u = lib->bonds[2 * (b0 + e)], v = lib->bonds[2 * (b0 + e) + 1];
        if (deg[u] < 2 || deg[v] < 2) { L->status = OR_LIG_TERMINAL_ROT; return L->status; }
        nrot++;
    }
    if (nrot > OR_MAX_TORS) { L->status = OR_LIG_NTORSIONS; return L->status; }

    /* reference conformer: input coordinates minus their unweighted mean */
    double c[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) c[d] += (double)lib->xyz[3 * (a0 + i) + d];
    for (int d = 0; d < 3; ++d) c[d] /= n;
    for (int i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) L->xref[i][d] = (double)lib->xyz[3 * (a0 + i) + d] - c[d];
        L->type[i] = lib->type[a0 + i];
    }

    /* rigid fragments: connected components of the non-rotatable bonds */
    int frag[OR_MAX_ATOMS];
    for (int i = 0; i < n; ++i) frag[i] = -1;
    int n_frag = 0, best_frag = -1, best_size = 0;
    for (int s = 0; s < n; ++s) {
        if (frag[s] >= 0) continue;
        int stack[OR_MAX_ATOMS], sp = 0, size = 0;
        frag[s] = n_frag;
        stack[sp++] = s;
        while (sp) {
            int x = stack[--sp];
            size++;
            for (int e = 0; e < nb; ++e) {
                if (lib->rot[b0 + e]) continue;
                int u = lib->bonds[2 * (b0 + e)], v = lib->bonds[2 * (b0 + e) + 1];
                int y = u == x ? v : (v == x ? u : -1);
                if (y >= 0 && frag[y] < 0) { frag[y] = n_frag; stack[sp++] = y; }
            }
        }
        /* fragments are discovered in increasing order of their lowest atom index,
           so a strict > keeps the lowest-index fragment among equal sizes */
        if (size > best_size) { best_size = size; best_frag = n_frag; }
        n_frag++;
    }
    for (int i = 0; i < n; ++i) L->core[i] = frag[i] == best_frag;

    /* torsions, oriented away from the core */
    int cnt = 0, msize[OR_MAX_TORS];
    int ta[OR_MAX_TORS], tb[OR_MAX_TORS], tbond[OR_MAX_TORS];
    unsigned char mv[OR_MAX_TORS][OR_MAX_ATOMS];
    for (int e = 0; e < nb; ++e) {
        if (!lib->rot[b0 + e]) continue;
        int u = lib->bonds[2 * (b0 + e)], v = lib->bonds[2 * (b0 + e) + 1];
        unsigned char side_v[OR_MAX_ATOMS];
        reach(n, deg, nbr, v, u, v, NULL, side_v);
        int core_on_v = 0;
        for (int i = 0; i < n; ++i) core_on_v |= (L->core[i] && side_v[i]);
        if (core_on_v) { /* core lies on v's side: v is the axis root, u's side moves */
            ta[cnt] = v; tb[cnt] = u;
            for (int i = 0; i < n; ++i) mv[cnt][i] = !side_v[i];
        } else {
            ta[cnt] = u; tb[cnt] = v;
            for (int i = 0; i < n; ++i) mv[cnt][i] = side_v[i];
        }
        msize[cnt] = 0;
        for (int i = 0; i < n; ++i) msize[cnt] += mv[cnt][i];
        tbond[cnt] = e;
        cnt++;
    }
    /* sweep order: descending moving-set size, ties by ascending bond index (stable) */
    int order[OR_MAX_TORS];
    for (int k = 0; k < cnt; ++k) order[k] = k;
    for (int k = 1; k < cnt; ++k) {
        int x = order[k], j = k - 1;
        while (j >= 0 && msize[order[j]] < msize[x]) { order[j + 1] = order[j]; j--; }
        order[j + 1] = x;
    }
    L->B = cnt;
    for (int k = 0; k < cnt; ++k) {
        int o = order[k];
        L->tor_a[k] = ta[o];
        L->tor_b[k] = tb[o];
        L->tor_bond[k] = tbond[o];
        memcpy(L->moving[k], mv[o], (size_t)n);
    }

    /* tree distances by breadth-first search from every atom, then the clash pairs */
    L->n_pairs = 0;
    for (int i = 0; i < n; ++i) {
        int dist[OR_MAX_ATOMS], queue[OR_MAX_ATOMS], qh = 0, qt = 0;
        for (int j = 0; j < n; ++j) dist[j] = -1;
        dist[i] = 0;
        queue[qt++] = i;
        while (qh < qt) {
            int x = queue[qh++];
            for (int q = 0; q < deg[x]; ++q) {
                int y = nbr[x][q];
                if (dist[y] < 0) { dist[y] = dist[x] + 1; queue[qt++] = y; }
            }
        }
        for (int j = i + 1; j < n; ++j)
            if (dist[j] >= 3) {
                L->pair_i[L->n_pairs] = i;
                L->pair_j[L->n_pairs] = j;
                L->n_pairs++;
            }
    }
    L->status = OR_LIG_OK;
    return OR_LIG_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Score and search                                                                            */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    int32_t n_quat;
    const float *quat; /* [n_quat][4] (w, x, y, z), not necessarily normalised */
    int32_t n_trans;
    const float *trans; /* [n_trans][3] */
    int32_t n_steps;    /* S: torsion angles 2 pi s / S, s = 0..S-1 */
    double clash_cut, clash_w;
    int32_t sweep_top;  /* 0: every start gets the torsion sweeps; K > 0: only the K best rigid starts */
    int32_t passes;     /* greedy passes over the torsions (values below 1 count as 1) */
    int32_t restarts;   /* R: torsion restarts per rigid start (not combined with sweep_top) */
    const int32_t *init_steps; /* [R][16] initial turn of torsion k of restart r, in [0, S) */
} or_search;

/* Searched starts: (1 + R) Q T; start e is restart e / (Q T) of rigid start e mod (Q T). */
static int64_t or_n_starts(const or_search *s)
{
    return (int64_t)s->n_quat * s->n_trans * (1 + (s->restarts > 0 ? s->restarts : 0));
}

/*
 * Score of conformer X: the sum over atoms of the interpolated grid value of the
 * atom's type, plus clash_w * max(0, clash_cut - d)^2 over the clash pairs.
 */
double or_score(const or_lig *L, const double X[][3], const or_frame *f, const float *G, const or_search *s)
{
    double e = 0.0;
    for (int i = 0; i < L->n; ++i) e += or_lookup(f, G, L->type[i], X[i]);
    for (int p = 0; p < L->n_pairs; ++p) {
        const double *a = X[L->pair_i[p]], *b = X[L->pair_j[p]];
        double d = sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2]));
        if (d < s->clash_cut) e += s->clash_w * (s->clash_cut - d) * (s->clash_cut - d);
    }
    return e;
}

/* Rigid start p = iq * n_trans + it: X = R(q_iq) Xref + t_it (p is taken modulo Q T, so a
   searched start e gives its rigid start). */
void or_place(const or_lig *L, const or_search *s, int p, double X[][3])
{
    p %= s->n_quat * s->n_trans;
    int iq = p / s->n_trans, it = p % s->n_trans;
    double q[4] = {s->quat[4 * iq], s->quat[4 * iq + 1], s->quat[4 * iq + 2], s->quat[4 * iq + 3]};
    double Rm[9];
    or_quat_matrix(q, Rm);
    for (int i = 0; i < L->n; ++i)
        for (int d = 0; d < 3; ++d)
            X[i][d] = Rm[3 * d] * L->xref[i][0] + Rm[3 * d + 1] * L->xref[i][1] + Rm[3 * d + 2] * L->xref[i][2] +
                      (double)s->trans[3 * it + d];
}

/* Turns torsion k of conformer X by step `step`: the moving atoms rotate about the current a -> b axis. */
void or_turn(const or_lig *L, const or_search *s, int k, int step, const double X[][3], double Y[][3])
{
    const double *xa = X[L->tor_a[k]], *xb = X[L->tor_b[k]];
    double u[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
    double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int d = 0; d < 3; ++d) u[d] /= un;
    double th = 2.0 * M_PI * step / s->n_steps;
    for (int i = 0; i < L->n; ++i) {
        if (!L->moving[k][i]) { memcpy(Y[i], X[i], sizeof(Y[i])); continue; }
        double v[3] = {X[i][0] - xa[0], X[i][1] - xa[1], X[i][2] - xa[2]}, r[3];
        or_rodrigues(u, th, v, r);
        for (int d = 0; d < 3; ++d) Y[i][d] = xa[d] + r[d];
    }
}

/*
 * The conformer searched start e begins from: rigid start e mod (Q T), then, for restart
 * r = e / (Q T) >= 1, each torsion k turned by init_steps[r - 1][k] in sweep order (a zero turn
 * leaves the torsion as it is).  steps[k] receives that initial turn (0 for r = 0).
 */
static void or_start(const or_lig *L, const or_search *s, int e, double X[][3], int steps[])
{
    double Y[OR_MAX_ATOMS][3];
    const int r = e / (s->n_quat * s->n_trans);
    or_place(L, s, e, X);
    for (int k = 0; k < L->B; ++k) {
        steps[k] = r > 0 ? s->init_steps[(r - 1) * OR_MAX_TORS + k] : 0;
        if (steps[k] == 0) continue;  /* no turn: the torsion is left as it is */
        or_turn(L, s, k, steps[k], (const double(*)[3])X, Y);
        memcpy(X, Y, sizeof(double) * 3 * L->n);
    }
}

/*
 * Greedy search from searched start p (a rigid start, or a torsion restart of one: or_start):
 * for each torsion in sweep order, score the conformer turned by every step, keep the lowest
 * (ties to the lowest step), and move on with that conformer; the whole pass over the torsions
 * is made s->passes times.  Returns the final score.  steps[k] receives torsion k's total turn,
 * its initial turn plus its chosen steps over the passes, modulo S (a turn changes only its own
 * torsion angle, so the final conformer is the rigid start's with each torsion turned once by its
 * total); min_gap (may be NULL) the smallest relative decision gap met,
 * (second-lowest - lowest) / max(1, |lowest|), +inf if there was no decision.
 */
double or_greedy(const or_lig *L, const or_frame *f, const float *G, const or_search *s, int p, int steps[],
                 double *min_gap)
{
    double X[OR_MAX_ATOMS][3], Y[OR_MAX_ATOMS][3], Best[OR_MAX_ATOMS][3];
    double gap = INFINITY;
    const int passes = s->passes > 1 ? s->passes : 1;
    or_start(L, s, p, X, steps);
    for (int pass = 0; pass < passes; ++pass)
    for (int k = 0; k < L->B; ++k) {
        double e1 = INFINITY, e2 = INFINITY;
        int s1 = 0;
        for (int st = 0; st < s->n_steps; ++st) {
            or_turn(L, s, k, st, (const double(*)[3])X, Y);
            double e = or_score(L, (const double(*)[3])Y, f, G, s);
            if (e < e1) { e2 = e1; e1 = e; s1 = st; memcpy(Best, Y, sizeof(double) * 3 * L->n); }
            else if (e < e2) e2 = e;
        }
        double g = (e2 - e1) / (fabs(e1) > 1.0 ? fabs(e1) : 1.0);
        if (g < gap) gap = g;
        steps[k] = (steps[k] + s1) % s->n_steps;
        memcpy(X, Best, sizeof(double) * 3 * L->n);
    }
    if (min_gap) *min_gap = gap;
    return or_score(L, (const double(*)[3])X, f, G, s);
}

/* Score of the explicit pose (start p, steps[k] for each torsion in sweep order: the total turns
   from the rigid start p mod Q T). */
double or_pose_score(const or_lig *L, const or_frame *f, const float *G, const or_search *s, int p,
                     const int32_t steps[])
{
    double X[OR_MAX_ATOMS][3], Y[OR_MAX_ATOMS][3];
    or_place(L, s, p, X);
    for (int k = 0; k < L->B; ++k) {
        or_turn(L, s, k, steps[k], (const double(*)[3])X, Y);
        memcpy(X, Y, sizeof(double) * 3 * L->n);
    }
    return or_score(L, (const double(*)[3])X, f, G, s);
}

/* ------------------------------------------------------------------------------------------ */
/* Batch entry points (ctypes)                                                                 */
/* ------------------------------------------------------------------------------------------ */

/* Topology of ligand l, flattened for inspection by tests. */
int or_topology(const or_library *lib, int64_t l, int32_t *status, int32_t *B, int32_t *tor_a, int32_t *tor_b,
                int32_t *tor_bond, uint8_t *moving /* [16][128] */, uint8_t *core /* [128] */, int32_t *n_pairs,
                int32_t *pairs /* [8128][2] */, double *xref /* [128][3] */)
{
    or_lig *L = (or_lig *)malloc(sizeof(or_lig));
    or_ligand(lib, l, L);
    *status = L->status;
    *B = L->B;
    *n_pairs = L->status == OR_LIG_OK ? L->n_pairs : 0;
    if (L->status == OR_LIG_OK) {
        for (int k = 0; k < L->B; ++k) {
            tor_a[k] = L->tor_a[k];
            tor_b[k] = L->tor_b[k];
            tor_bond[k] = L->tor_bond[k];
            for (int i = 0; i < L->n; ++i) moving[k * OR_MAX_ATOMS + i] = L->moving[k][i];
        }
        for (int i = 0; i < L->n; ++i) {
            core[i] = L->core[i];
            for (int d = 0; d < 3; ++d) xref[3 * i + d] = L->xref[i][d];
        }
        for (int p = 0; p < L->n_pairs; ++p) { pairs[2 * p] = L->pair_i[p]; pairs[2 * p + 1] = L->pair_j[p]; }
    }
    free(L);
    return 0;
}

/* Status code of every ligand of the library. */
int or_status(const or_library *lib, int64_t n_lig, int32_t *status)
{
#pragma omp parallel
    {
        or_lig *L = (or_lig *)malloc(sizeof(or_lig));
#pragma omp for schedule(dynamic, 16)
        for (int64_t l = 0; l < n_lig; ++l) status[l] = or_ligand(lib, l, L);
        free(L);
    }
    return 0;
}

/* Loads the selected ligands; returns a malloc'd array of n_sel ligands. */
static or_lig *load_selection(const or_library *lib, int32_t n_sel, const int64_t *sel)
{
    or_lig *Ls = (or_lig *)malloc(sizeof(or_lig) * (size_t)(n_sel > 0 ? n_sel : 1));
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t i = 0; i < n_sel; ++i) or_ligand(lib, sel[i], &Ls[i]);
    return Ls;
}

/* Orders (score, start) pairs: lower score first, ties to the lower start. */
typedef struct {
    double e;
    int32_t p;
} or_keyed;

static int or_keyed_cmp(const void *a, const void *b)
{
    const or_keyed *x = (const or_keyed *)a, *y = (const or_keyed *)b;
    if (x->e < y->e) return -1;
    if (x->e > y->e) return 1;
    return (x->p > y->p) - (x->p < y->p);
}

/*
 * Docks the selected ligands.  The greedy search is run from every rigid start (the
 * multiple restarts), or, with s->sweep_top = K in [1, Q*T), only from the K starts
 * whose rigid pose scores lowest (ties to the lower start); with s->restarts = R > 0 also
 * from R torsion restarts of every rigid start (or_start), (1 + R) Q T searched starts.
 * The ligand's result is its best searched start, ties to the lowest start index.
 * Ligands with a non-OK status get +inf and start -1.  Optional per-start outputs: finals
 * [n_sel][N] (+inf for starts not searched), start_steps [n_sel][N][16], start_gap
 * [n_sel][N], N the number of searched starts.
 */
int or_dock(const or_frame *f, const float *G, const or_library *lib, const or_search *s, int32_t n_sel,
            const int64_t *sel, double *best, int32_t *best_p, int32_t *best_steps, int32_t *status,
            double *finals, int32_t *start_steps, double *start_gap)
{
    or_lig *Ls = load_selection(lib, n_sel, sel);
    int64_t QT = or_n_starts(s);  /* searched starts, restarts included */
    size_t cells = (size_t)(n_sel * QT > 0 ? n_sel * QT : 1);
    double *fin = (double *)malloc(sizeof(double) * cells);
    int32_t *stp = (int32_t *)malloc(sizeof(int32_t) * OR_MAX_TORS * cells);
    uint8_t *searched = (uint8_t *)malloc(cells);
    const int top = s->restarts <= 0 && s->sweep_top > 0 && s->sweep_top < QT;
    memset(searched, top ? 0 : 1, cells);
    if (top) {
        /* rigid scores of every start, then the K lowest per ligand */
        or_keyed *rk = (or_keyed *)malloc(sizeof(or_keyed) * cells);
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t w = 0; w < (int64_t)n_sel * QT; ++w) {
            int32_t i = (int32_t)(w / QT);
            double X[OR_MAX_ATOMS][3];
            rk[w].p = (int32_t)(w % QT);
            rk[w].e = INFINITY;
            if (Ls[i].status != OR_LIG_OK) continue;
            or_place(&Ls[i], s, rk[w].p, X);
            rk[w].e = or_score(&Ls[i], (const double(*)[3])X, f, G, s);
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int32_t i = 0; i < n_sel; ++i) {
            qsort(rk + (size_t)i * QT, (size_t)QT, sizeof(or_keyed), or_keyed_cmp);
            for (int k = 0; k < s->sweep_top; ++k) searched[(size_t)i * QT + rk[(size_t)i * QT + k].p] = 1;
        }
        free(rk);
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t w = 0; w < (int64_t)n_sel * QT; ++w) {
        int32_t i = (int32_t)(w / QT);
        int p = (int)(w % QT);
        for (int k = 0; k < OR_MAX_TORS; ++k) stp[w * OR_MAX_TORS + k] = 0;
        if (start_gap) start_gap[w] = INFINITY;
        if (Ls[i].status != OR_LIG_OK || !searched[w]) { fin[w] = INFINITY; continue; }
        int steps[OR_MAX_TORS] = {0};
        double gap;
        fin[w] = or_greedy(&Ls[i], f, G, s, p, steps, &gap);
        for (int k = 0; k < OR_MAX_TORS; ++k) stp[w * OR_MAX_TORS + k] = steps[k];
        if (start_gap) start_gap[w] = gap;
    }
    for (int32_t i = 0; i < n_sel; ++i) {
        status[i] = Ls[i].status;
        double b = INFINITY;
        int bp = -1;
        for (int64_t p = 0; p < QT; ++p)
            if (fin[i * QT + p] < b) { b = fin[i * QT + p]; bp = (int)p; }
        best[i] = b;
        best_p[i] = bp;
        for (int k = 0; k < OR_MAX_TORS; ++k)
            best_steps[i * OR_MAX_TORS + k] = bp >= 0 ? stp[(i * QT + bp) * OR_MAX_TORS + k] : 0;
        if (finals) memcpy(finals + i * QT, fin + i * QT, sizeof(double) * (size_t)QT);
        if (start_steps) memcpy(start_steps + i * QT * OR_MAX_TORS, stp + i * QT * OR_MAX_TORS,
                                sizeof(int32_t) * OR_MAX_TORS * (size_t)QT);
    }
    free(searched);
    free(stp);
    free(fin);
    free(Ls);
    return 0;
}

/* Greedy pass of single (ligand, start) pairs: final score, chosen steps and min decision gap. */
int or_greedy_starts(const or_frame *f, const float *G, const or_library *lib, const or_search *s, int64_t n,
                     const int64_t *lig, const int32_t *start, double *final, int32_t *steps, double *gap)
{
#pragma omp parallel
    {
        or_lig *L = (or_lig *)malloc(sizeof(or_lig));
        int64_t cur = -1;
#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < n; ++w) {
            if (lig[w] != cur) { or_ligand(lib, lig[w], L); cur = lig[w]; }
            int st[OR_MAX_TORS] = {0};
            double g = INFINITY;
            final[w] = L->status == OR_LIG_OK ? or_greedy(L, f, G, s, start[w], st, &g) : INFINITY;
            for (int k = 0; k < OR_MAX_TORS; ++k) steps[w * OR_MAX_TORS + k] = st[k];
            if (gap) gap[w] = g;
        }
        free(L);
    }
    return 0;
}

/* Scores explicit pose descriptors (ligand, start, steps in sweep order). */
int or_score_poses(const or_frame *f, const float *G, const or_library *lib, const or_search *s, int64_t n,
                   const int64_t *lig, const int32_t *start, const int32_t *steps, double *out)
{
#pragma omp parallel
    {
        or_lig *L = (or_lig *)malloc(sizeof(or_lig));
        int64_t cur = -1;
#pragma omp for schedule(dynamic, 16)
        for (int64_t w = 0; w < n; ++w) {
            if (lig[w] != cur) { or_ligand(lib, lig[w], L); cur = lig[w]; }
            out[w] = L->status == OR_LIG_OK ? or_pose_score(L, f, G, s, start[w], steps + w * OR_MAX_TORS) : INFINITY;
        }
        free(L);
    }
    return 0;
}

/*
 * Follows a given path (searched start, total turns) and, at every torsion, reports the score
 * of the given step (the total less the start's initial turn) and the lowest score over all
 * steps from the same conformer; used to check that each decision of another implementation
 * is a (near-)argmin.  One pass.
 */
int or_replay(const or_frame *f, const float *G, const or_library *lib, const or_search *s, int64_t n,
              const int64_t *lig, const int32_t *start, const int32_t *steps, double *e_given, double *e_min,
              double *final)
{
#pragma omp parallel
    {
        or_lig *L = (or_lig *)malloc(sizeof(or_lig));
        double X[OR_MAX_ATOMS][3], Y[OR_MAX_ATOMS][3];
#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < n; ++w) {
            or_ligand(lib, lig[w], L);
            for (int k = 0; k < OR_MAX_TORS; ++k) { e_given[w * OR_MAX_TORS + k] = NAN; e_min[w * OR_MAX_TORS + k] = NAN; }
            if (L->status != OR_LIG_OK) { final[w] = INFINITY; continue; }
            int init[OR_MAX_TORS];
            or_start(L, s, start[w], X, init);
            for (int k = 0; k < L->B; ++k) {
                double emin = INFINITY, eg = NAN;
                /* the given steps are total turns; the decision is the turn on top of the start's */
                int sg = ((steps[w * OR_MAX_TORS + k] - init[k]) % s->n_steps + s->n_steps) % s->n_steps;
                for (int st = 0; st < s->n_steps; ++st) {
                    or_turn(L, s, k, st, (const double(*)[3])X, Y);
                    double e = or_score(L, (const double(*)[3])Y, f, G, s);
                    if (e < emin) emin = e;
                    if (st == sg) eg = e;
                }
                e_given[w * OR_MAX_TORS + k] = eg;
                e_min[w * OR_MAX_TORS + k] = emin;
                or_turn(L, s, k, sg, (const double(*)[3])X, Y);
                memcpy(X, Y, sizeof(double) * 3 * L->n);
            }
            final[w] = or_score(L, (const double(*)[3])X, f, G, s);
        }
        free(L);
    }
    return 0;
}

/*
 * Exhaustive search of ligand l: the lowest score over every start and every
 * combination of steps (S^B per start).  Ties go to the lowest start, then the
 * lexicographically lowest step vector.  Only for tiny ligands.
 */
int or_exhaustive(const or_frame *f, const float *G, const or_library *lib, const or_search *s, int64_t l,
                  double *best, int32_t *best_p, int32_t *best_steps)
{
    or_lig *L = (or_lig *)malloc(sizeof(or_lig));
    or_ligand(lib, l, L);
    *best = INFINITY;
    *best_p = -1;
    if (L->status != OR_LIG_OK) { free(L); return L->status; }
    int64_t combos = 1;
    for (int k = 0; k < L->B; ++k) combos *= s->n_steps;
    int64_t QT = (int64_t)s->n_quat * s->n_trans;
    double *sc = (double *)malloc(sizeof(double) * (size_t)(QT * combos));
#pragma omp parallel for schedule(static)
    for (int64_t w = 0; w < QT * combos; ++w) {
        int p = (int)(w / combos);
        int64_t c = w % combos;
        int32_t st[OR_MAX_TORS] = {0};
        for (int k = L->B - 1; k >= 0; --k) { st[k] = (int32_t)(c % s->n_steps); c /= s->n_steps; }
        sc[w] = or_pose_score(L, f, G, s, p, st);
    }
    int64_t bw = -1;
    for (int64_t w = 0; w < QT * combos; ++w)
        if (sc[w] < *best) { *best = sc[w]; bw = w; }
    if (bw >= 0) {
        *best_p = (int32_t)(bw / combos);
        int64_t c = bw % combos;
        for (int k = L->B - 1; k >= 0; --k) { best_steps[k] = (int32_t)(c % s->n_steps); c /= s->n_steps; }
    }
    free(sc);
    free(L);
    return 0;
}

/* Interpolated grid value plus restraint at arbitrary points (for pinning tests). */
int or_lookup_points(const or_frame *f, const float *G, int64_t n, const int32_t *t, const double *x, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = or_lookup(f, G, t[i], x + 3 * i);
    return 0;
}

/* Grid values at sampled nodes (t, i, j, k), FP64 before the FP32 store. */
int or_grid_nodes(const or_frame *f, const or_potential *pot, const float *prot_xyz, const int32_t *prot_type,
                  int32_t n_prot, int64_t n, const int32_t *tijk, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t w = 0; w < n; ++w)
        out[w] = or_grid_node(f, pot, prot_xyz, prot_type, n_prot, tijk[4 * w], tijk[4 * w + 1], tijk[4 * w + 2],
                              tijk[4 * w + 3]);
    return 0;
}

/* Score of explicit conformers X [n][3] of ligand l (any coordinates; pins the score definition). */
int or_score_conformer(const or_frame *f, const float *G, const or_library *lib, const or_search *s, int64_t l,
                       const double *X, double *out)
{
    or_lig *L = (or_lig *)malloc(sizeof(or_lig));
    or_ligand(lib, l, L);
    *out = L->status == OR_LIG_OK ? or_score(L, (const double(*)[3])X, f, G, s) : INFINITY;
    free(L);
    return 0;
}

/* Applies start p and the given steps, returning the conformer (pins the motion definitions). */
int or_pose_coords(const or_library *lib, const or_search *s, int64_t l, int32_t p, const int32_t *steps,
                   int32_t upto, double *X_out)
{
    or_lig *L = (or_lig *)malloc(sizeof(or_lig));
    or_ligand(lib, l, L);
    double X[OR_MAX_ATOMS][3], Y[OR_MAX_ATOMS][3];
    or_place(L, s, p, X);
    for (int k = 0; k < L->B && k < upto; ++k) {
        or_turn(L, s, k, steps[k], (const double(*)[3])X, Y);
        memcpy(X, Y, sizeof(double) * 3 * L->n);
    }
    memcpy(X_out, X, sizeof(double) * 3 * L->n);
    free(L);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Pose filtering and rescoring                                                                */
/* ------------------------------------------------------------------------------------------ */

/*
 * Rescoring pair energy: the same 6-12 well as the grid potential, and Coulomb with the
 * distance-dependent dielectric 4 r in place of the constant 4 (coulomb_k already holds the
 * factor 1/4): coulomb_k q_a q_b / r'^2; r floored at r_min.
 */
double or_rescore_pair(double r, int a, int b, const or_potential *pot)
{
    double rt = r > pot->r_min ? r : pot->r_min;
    double r0 = pot->R[a] + pot->R[b];
    double eps = sqrt(pot->eps[a] * pot->eps[b]);
    double s6 = pow(r0 / rt, 6.0);
    return eps * (s6 * s6 - 2.0 * s6) + pot->coulomb_k * pot->q[a] * pot->q[b] / (rt * rt);
}

/*
 * Rescoring of conformer X: for every ligand atom the sum of or_rescore_pair over the protein
 * atoms at the atom's own position (no grid, no interpolation), capped at pot->cap, plus the
 * intra-ligand clash term of the docking score.
 */
double or_rescore(const or_lig *L, const double X[][3], const or_potential *pot, const float *prot_xyz,
                  const int32_t *prot_type, int32_t n_prot, const or_search *s)
{
    double e = 0.0;
    for (int i = 0; i < L->n; ++i) {
        double sum = 0.0;
        for (int32_t p = 0; p < n_prot; ++p) {
            double dx = X[i][0] - (double)prot_xyz[3 * p], dy = X[i][1] - (double)prot_xyz[3 * p + 1];
            double dz = X[i][2] - (double)prot_xyz[3 * p + 2];
            sum += or_rescore_pair(sqrt(dx * dx + dy * dy + dz * dz), L->type[i], prot_type[p], pot);
        }
        e += sum < pot->cap ? sum : pot->cap;
    }
    for (int q = 0; q < L->n_pairs; ++q) {
        const double *a = X[L->pair_i[q]], *b = X[L->pair_j[q]];
        double d = sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2]));
        if (d < s->clash_cut) e += s->clash_w * (s->clash_cut - d) * (s->clash_cut - d);
    }
    return e;
}

/* Root mean square deviation of two conformers of one ligand, atom by atom, no superposition. */
double or_rmsd(int n, const double X[][3], const double Y[][3])
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) s += (X[i][d] - Y[i][d]) * (X[i][d] - Y[i][d]);
    return sqrt(s / n);
}

/*
 * Filters and rescores poses of ligand l given in docking order (start[i], steps[i][16]): a pose
 * is kept unless an earlier kept pose lies within rmsd_min of it; kept poses get or_rescore,
 * dropped ones NaN.  nearest[i] is the RMSD to the closest earlier kept pose (+inf if none).
 * Poses with start < 0 are absent (dropped, NaN, +inf).
 */
int or_filter_rescore(const or_potential *pot, const float *prot_xyz, const int32_t *prot_type, int32_t n_prot,
                      const or_library *lib, const or_search *s, int64_t l, int32_t n_poses, const int32_t *start,
                      const int32_t *steps, double rmsd_min, int32_t *kept, double *rescore, double *nearest)
{
    or_lig *L = (or_lig *)malloc(sizeof(or_lig));
    or_ligand(lib, l, L);
    double(*P)[OR_MAX_ATOMS][3] = malloc(sizeof(double) * OR_MAX_ATOMS * 3 * (size_t)(n_poses > 0 ? n_poses : 1));
    double Y[OR_MAX_ATOMS][3];
    for (int32_t i = 0; i < n_poses; ++i) {
        kept[i] = 0;
        rescore[i] = NAN;
        nearest[i] = INFINITY;
        if (L->status != OR_LIG_OK || start[i] < 0) continue;
        or_place(L, s, start[i], P[i]);
        for (int k = 0; k < L->B; ++k) {
            or_turn(L, s, k, steps[i * OR_MAX_TORS + k], (const double(*)[3])P[i], Y);
            memcpy(P[i], Y, sizeof(double) * 3 * L->n);
        }
        for (int32_t j = 0; j < i; ++j) {
            if (!kept[j]) continue;
            double r = or_rmsd(L->n, (const double(*)[3])P[i], (const double(*)[3])P[j]);
            if (r < nearest[i]) nearest[i] = r;
        }
        kept[i] = !(nearest[i] < rmsd_min);
        if (kept[i]) rescore[i] = or_rescore(L, (const double(*)[3])P[i], pot, prot_xyz, prot_type, n_prot, s);
    }
    free(P);
    free(L);
    return 0;
}

/* Rescoring of explicit conformers X [n][3] of ligand l (any coordinates; pins the definition). */
int or_rescore_conformer(const or_potential *pot, const float *prot_xyz, const int32_t *prot_type, int32_t n_prot,
                         const or_library *lib, const or_search *s, int64_t l, const double *X, double *out)
{
    or_lig *L = (or_lig *)malloc(sizeof(or_lig));
    or_ligand(lib, l, L);
    *out = L->status == OR_LIG_OK ? or_rescore(L, (const double(*)[3])X, pot, prot_xyz, prot_type, n_prot, s)
                                  : INFINITY;
    free(L);
    return 0;
}

void or_quat_matrix_c(const double *q, double *Rm) { or_quat_matrix(q, Rm); }
void or_rodrigues_c(const double *u, double th, const double *v, double *out) { or_rodrigues(u, th, v, out); }

/* Thread count of the batch entry points (OpenMP); not part of the method. */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_get_threads(void) { return omp_get_max_threads(); }
