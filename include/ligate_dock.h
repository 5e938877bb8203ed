/*
 * ligate_dock.h - C ABI of the MI355X docking screen.
 *
 * The operation (paper §2, "LIGATE CADD Workflow"): rank a virtual ligand
 * library against one rigid binding site.  A receptor is prepared once as
 * per-atom-type interaction grids; ligands stream through a pose search with
 * multiple restarts scored by a geometric function; a ligand's score is the
 * score of its best pose; the library is ranked and the strongest binders are
 * returned.  Batching of ligands of uneven size follows §3.3 ("LiGen
 * Autotuning", the batch redesign).
 *
 * Conventions shared by every call:
 *  - Pointers named d_* are device (HIP) memory, h_* are host memory.  The
 *    caller owns every buffer; the library never allocates device memory.
 *    Scratch comes in through d_ws, sized by a query: pass d_ws == NULL and the
 *    required size is written to *ws_bytes (nothing is enqueued).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *    enqueues work on it: no device allocation, no host synchronisation, no
 *    hipMemset, so every call can be captured into a hipGraph.
 *  - Argument errors are returned synchronously (negative status) before any
 *    work is enqueued.  Data-dependent problems with a ligand (a bond graph that
 *    is not a tree, ...) are not call failures: they are reported per ligand in
 *    d_status and such a ligand scores +inf.
 *  - A HIP launch failure returns DOCK_ERR_HIP; dock_last_error() has detail.
 *  - Calls are not thread-safe on one stream; different streams are independent.
 */
#ifndef LIGATE_DOCK_H
#define LIGATE_DOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- call status ------------------------------------------------------------------------- */
#define DOCK_OK 0
#define DOCK_ERR_INVALID_ARG (-1) /* null pointer, bad count or size, inconsistent descriptor */
#define DOCK_ERR_LIMIT (-2)       /* a documented limit below is exceeded */
#define DOCK_ERR_HIP (-3)         /* the HIP runtime reported an error */
#define DOCK_ERR_WORKSPACE (-4)   /* d_ws / d_pack smaller than the queried size */

/* ---- per-ligand status (d_status), checked in this order; the first failure is reported ---- */
#define DOCK_LIG_OK 0
#define DOCK_LIG_NATOMS 1       /* n < 1 or n > DOCK_MAX_ATOMS */
#define DOCK_LIG_TYPE 2         /* an atom type >= n_types */
#define DOCK_LIG_NBONDS 3       /* bond count != n - 1 */
#define DOCK_LIG_BOND_INDEX 4   /* bond endpoint outside [0, n) or a self bond */
#define DOCK_LIG_DEGREE 5       /* an atom with more than 4 bonds */
#define DOCK_LIG_NOT_TREE 6     /* the bond graph is not connected */
#define DOCK_LIG_TERMINAL_ROT 7 /* a rotatable bond with an endpoint of degree 1 */
#define DOCK_LIG_NTORSIONS 8    /* more than DOCK_MAX_TORSIONS rotatable bonds */

/* ---- limits ------------------------------------------------------------------------------- */
#define DOCK_MAX_ATOMS 128
#define DOCK_MAX_TORSIONS 16
#define DOCK_MAX_TYPES 32
#define DOCK_MAX_STEPS 1024
#define DOCK_MAX_TOP_STARTS 8192 /* starts ranked per ligand when sweep_top selects */
#define DOCK_MAX_PASSES 16
#define DOCK_MAX_RESTARTS 64     /* torsion restarts per rigid start */

#define DOCK_LAYOUT_LINEAR 0     /* grids [t][z][y][x], FP32, x fastest */
#define DOCK_LAYOUT_XY4 1        /* per node a 16-byte record of its z plane: G00 = G(x, y),
                                    dX = G(x+1, y) - G00, dY = G(x, y+1) - G00,
                                    dXY = (G(x+1, y+1) - G(x, y+1)) - dX (differences rounded to
                                    FP32; indices beyond the last node wrap to 0), stored as
                                    [t][z/2][y/2][x][z&1][y&1] with dimensions rounded up to even,
                                    so that a 128-byte line holds 2 x 2 x 2 records; about 4x the
                                    memory, and a trilinear lookup reads two records, mostly from
                                    one line.  Requires (nx rounded up to even) * ceil(ny / 2)
                                    <= 2^18 */
#define DOCK_BOUNDARY_CLAMP 0    /* clamp into the box + w_out * |x - clamp(x)|^2 */
#define DOCK_BOUNDARY_PERIODIC 1 /* indices wrap modulo the grid size */

/*
 * Receptor grid frame.  Node (i, j, k) sits at origin + spacing * (i, j, k);
 * 2 <= nx, ny, nz; nx*ny*nz < 2^24; 1 <= n_types <= DOCK_MAX_TYPES; spacing > 0;
 * the grids of all types together below 2^31 bytes.  Lookups give the same
 * values in either layout; a layout is fixed when the grids are built.
 */
typedef struct {
    int32_t nx, ny, nz, n_types;
    float origin[3];
    float spacing;  /* Angstrom */
    int32_t layout; /* DOCK_LAYOUT_LINEAR or DOCK_LAYOUT_XY4 */
    int32_t boundary;
    float w_out;    /* restraint weight for DOCK_BOUNDARY_CLAMP */
} dock_grid_desc;

/* Per atom type: radius R (Angstrom), well depth eps, partial charge q. */
typedef struct {
    double R, eps, q;
} dock_type_param;

/* Grid potential: values are capped at `cap`; distances floored at r_min; Coulomb constant / dielectric. */
typedef struct {
    double cap, r_min, coulomb_k;
} dock_potential;

/*
 * Pose search.  Rigid start p = iq * n_trans + it places the centred ligand
 * with quaternion d_quat[iq] (w, x, y, z; normalised by the library) and
 * translation d_trans[it]; then a greedy pass turns each torsion, in sweep
 * order, by the best of the n_steps angles 2 pi s / n_steps.  Search budget:
 * with sweep_top = K in [1, n_quat*n_trans) only the K starts whose rigid pose
 * scores lowest (FP32, ties to the lower start) get the greedy passes, which
 * needs n_quat*n_trans <= DOCK_MAX_TOP_STARTS; 0 or K >= n_quat*n_trans
 * searches from every start.  passes (0 or 1 = one; at most DOCK_MAX_PASSES)
 * repeats the pass over the torsions.  Torsion restarts: with restarts = R > 0
 * (not combined with sweep_top) the search also starts from R turned copies of
 * every rigid start; searched start e = r * n_quat*n_trans + p (r = 0 .. R) is
 * rigid start p with, for r >= 1, each torsion k first turned by
 * d_init_steps[r-1][k] in sweep order (a zero turn leaves it as it is).  The
 * caller draws the initial turns, in [0, n_steps).
 */
typedef struct {
    int32_t n_quat;
    const float *d_quat;  /* [n_quat][4], device */
    int32_t n_trans;
    const float *d_trans; /* [n_trans][3], device, Angstrom */
    int32_t n_steps;      /* 1 .. DOCK_MAX_STEPS */
    float clash_cut;      /* pairs three or more bonds apart closer than this clash */
    float clash_w;        /* clash weight: clash_w * (clash_cut - d)^2 */
    int32_t starts_per_item; /* rigid starts per work item; 0 = chosen by the library */
    int32_t waves_per_block; /* 1, 2, 4 or 8; 0 = chosen by the library */
    int32_t sweep_top;       /* 0 = every start; K = the K best rigid starts */
    int32_t passes;          /* greedy passes over the torsions; 0 = 1 */
    int32_t restarts;        /* R torsion restarts per rigid start, 0 .. DOCK_MAX_RESTARTS */
    const int32_t *d_init_steps; /* [R][16] initial turns, device; NULL when R = 0 */
} dock_search;

/* Size in bytes of the grids for descriptor g (paper §2: the target is prepared once,
 * before the library streams through). */
int dock_grid_bytes(const dock_grid_desc *g, size_t *bytes);

/*
 * Paper §2: the workflow is structure based, scoring ligands against the 3D
 * shape of the target's binding site; the receptor side of that score is
 * tabulated once per pocket.  The functional form is this library's reading
 * (the paper calls the docking score geometric and gives no formula).
 * Builds the receptor grids: for every ligand atom type t and node x,
 * G_t(x) = min(cap, sum_j E(t, type_j, |x - p_j|)) with
 * E(a, b, r) = sqrt(eps_a eps_b) [(r0/r')^12 - 2 (r0/r')^6] + coulomb_k q_a q_b / r',
 * r0 = R_a + R_b, r' = max(r, r_min); summed in FP64, stored in FP32.
 * d_prot_xyz: [n_prot][3] FP32; d_prot_type: [n_prot] in [0, n_types);
 * h_params: [n_types] host; d_grids: dock_grid_bytes(g) bytes.
 */
int dock_build_grids(const dock_grid_desc *g, const float *d_prot_xyz, const int32_t *d_prot_type, int32_t n_prot,
                     const dock_type_param *h_params, const dock_potential *pot, float *d_grids, void *stream);

/*
 * Paper §2 (the first component computes each ligand's 3D atom placement for
 * the later ones) and §3.3 (ligands are grouped by atom and rotatable-bond
 * counts before the batched GPU kernels).
 * Packs a ligand library for the screen: centres each input conformer on its
 * unweighted centroid, stores coordinates as SoA, validates the bond tree,
 * finds the core (largest rigid fragment; ties to the one holding the lowest
 * atom index), orients each rotatable bond away from the core with a 128-bit
 * moving-atom mask, orders torsions for the sweep (larger moving sets first,
 * ties by bond index) and records, per atom, the atoms fewer than three bonds
 * away (excluded from the clash term).
 * Input (device, CSR): d_atom_off [n_lig+1], d_xyz [n_atoms_total][3] FP32,
 * d_type [n_atoms_total], d_bond_off [n_lig+1], d_bonds [n_bonds][2] (local
 * atom indices), d_rot [n_bonds] (nonzero = rotatable).  n_atoms_total must be
 * d_atom_off[n_lig].  With d_pack == NULL the required size is written to
 * *pack_bytes; otherwise *pack_bytes is the size of d_pack.  d_status [n_lig]
 * receives DOCK_LIG_* codes.  The pack is opaque and device-resident.
 */
int dock_pack_ligands(const int32_t *d_atom_off, const float *d_xyz, const uint8_t *d_type,
                      const int32_t *d_bond_off, const int32_t *d_bonds, const uint8_t *d_rot, int32_t n_lig,
                      int64_t n_atoms_total, int32_t n_types, void *d_pack, size_t *pack_bytes, int32_t *d_status,
                      void *stream);

/*
 * Paper §2: docking by a local search with multiple restarts, a geometric
 * score per pose, and a ligand scored as its best pose; §3.3: a batch of
 * ligand-protein pairs processed across the device at once, and the quality
 * knobs (starts, steps, passes, restarts) of the search.
 * Docks every packed ligand: the searched starts (every rigid start, or the
 * sweep_top best, and their torsion restarts), each followed by the greedy
 * torsion passes; per ligand the lowest final score wins, ties to the lowest
 * searched start.  With N = (1 + restarts) * n_quat*n_trans searched starts,
 * outputs, indexed by the ligand's position in the packed library:
 * d_best_score [n_lig] (+inf for a ligand whose status is not OK),
 * d_best_start [n_lig] (searched start e in [0, N); -1 if not OK),
 * d_best_steps [n_lig][16] (each torsion's total turn in sweep order: its
 * initial turn plus its chosen steps over the passes, modulo n_steps; a turn
 * changes only its own torsion angle, so the final pose is rigid start
 * e mod n_quat*n_trans with each torsion turned once by its total; unused
 * entries 0), optional d_start_scores [n_lig][N] (final score of every
 * searched start, +inf for starts not searched; NULL to skip), optional
 * d_start_steps [n_lig][N][16] (every searched start's totals; NULL to skip),
 * optional d_pose_count [1] (distinct poses scored: per docked ligand
 * N*(1 + passes*B*(n_steps-1)), or with sweep_top = K,
 * n_quat*n_trans + K*passes*B*(n_steps-1)).  n_lig and n_atoms_total must match
 * the pack.  Workspace: query with d_ws == NULL.
 */
int dock_screen(const dock_grid_desc *g, const float *d_grids, const void *d_pack, int32_t n_lig,
                int64_t n_atoms_total, const dock_search *s, float *d_best_score, int32_t *d_best_start,
                uint16_t *d_best_steps, float *d_start_scores, uint16_t *d_start_steps, uint64_t *d_pose_count,
                void *d_ws, size_t *ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under hipGraph capture,
 * tight serving loops, harnesses that forbid allocation): dock_screen with the
 * same arguments and outputs, minus the workspace.  Its scratch is a fixed
 * device array of DOCK_NOALLOC_SCRATCH_BYTES inside the library, one per GPU,
 * allocated when the library's code object is loaded and held until the
 * process ends; the call allocates nothing.  The scratch needed is that of
 * dock_screen's workspace query (about 25 bytes per ligand, plus 4 * sweep_top
 * per ligand with start selection); a screen needing more returns
 * DOCK_ERR_LIMIT before anything is enqueued.  Every call on one GPU shares that
 * GPU's array and clears what it needs on the device: calls that overlap on one
 * GPU (two streams, or two host threads) race and give undefined results; calls
 * in sequence on one stream are safe.  The first call on each device looks up
 * that device's array (a HIP symbol query, no allocation).
 */
#define DOCK_NOALLOC_SCRATCH_BYTES (32u << 20)
int dock_screen_noalloc(const dock_grid_desc *g, const float *d_grids, const void *d_pack, int32_t n_lig,
                        int64_t n_atoms_total, const dock_search *s, float *d_best_score, int32_t *d_best_start,
                        uint16_t *d_best_steps, float *d_start_scores, uint16_t *d_start_steps,
                        uint64_t *d_pose_count, void *stream);

/*
 * Paper §2: the poses the docking generates are filtered, and the survivors are
 * rescored with a function that adds physico-chemical information.
 * Pose filtering and rescoring after dock_screen.  For every packed ligand: the
 * n_keep searched starts with the lowest final scores in d_start_scores
 * (dock_screen's per-start output, [n_lig][N] with N = (1 + restarts) *
 * n_quat*n_trans as in dock_screen; ties to the lower start; +inf entries are
 * not taken), in that order, each rerun with the
 * screen's own code to recover its pose (its final equals the d_start_scores
 * entry bit for bit).  Walking them in that order, a pose is dropped when an
 * earlier kept pose lies within rmsd_min Angstrom of it (atom-by-atom RMSD, no
 * superposition); every kept pose is rescored at its atoms' own positions, in
 * FP64: per ligand atom min(cap, sum over the protein atoms of
 * sqrt(eps_a eps_b)[(r0/r')^12 - 2(r0/r')^6] + coulomb_k q_a q_b / r'^2)
 * (the grid potential with the distance-dependent dielectric 4r in place of 4,
 * no grid, no interpolation), plus the intra-ligand clash term.
 * g, d_grids, d_pack, n_lig, n_atoms_total, s: as for dock_screen (the same
 * search; N <= DOCK_MAX_TOP_STARTS).  Protein and potential: as
 * for dock_build_grids.  1 <= n_keep <= 16; rmsd_min >= 0 (Angstrom).
 * Outputs [n_lig][n_keep]: d_pose_start (-1 where there is no pose),
 * d_pose_steps [..][16] (total turns), d_pose_score (docking score, NaN where
 * no pose), d_pose_rescore (NaN where dropped or absent); [n_lig]:
 * d_best_rescore (lowest rescore, +inf if none), d_best_pose (its slot, ties
 * to the earlier slot; -1 if none).  Optional d_pose_xyz
 * [n_lig][n_keep][128][3] FP64 (the coordinates each kept pose was rescored
 * at; NULL to skip).  No workspace.
 */
int dock_rescore(const dock_grid_desc *g, const float *d_grids, const void *d_pack, int32_t n_lig,
                 int64_t n_atoms_total, const dock_search *s, const float *d_start_scores, const float *d_prot_xyz,
                 const int32_t *d_prot_type, int32_t n_prot, const dock_type_param *h_params,
                 const dock_potential *pot, int32_t n_keep, float rmsd_min, int32_t *d_pose_start,
                 uint16_t *d_pose_steps, float *d_pose_score, float *d_pose_rescore, float *d_best_rescore,
                 int32_t *d_best_pose, double *d_pose_xyz, void *stream);

/*
 * Paper §2: the screened library is ranked and a small set of the strongest
 * predicted binders is kept for the next stage.
 * Ranks scores: the k lowest, ties to the lower id, NaN ranked as +inf;
 * results in ascending order.  d_ids [n] (>= 0) or NULL for ids 0..n-1.
 * 1 <= k <= n < 2^31.  Workspace: query with d_ws == NULL.
 */
int dock_topk(const float *d_scores, const int32_t *d_ids, int64_t n, int32_t k, float *d_out_scores,
              int32_t *d_out_ids, void *d_ws, size_t *ws_bytes, void *stream);

/*
 * Paper §2: the molecules kept are those predicted to bind strongly to at least
 * one binding site of the targets.
 * Ranking over several binding sites (a ligand is as good as its best site):
 * d_scores [n_pockets][n] holds, row by row, dock_screen's d_best_score of the
 * same n ligands against each pocket; NaN counts as +inf.  d_best [n] receives
 * each ligand's lowest score and d_pocket [n] the row it came from (ties to the
 * lower row; -1 when every score is +inf).  dock_topk over d_best then ranks
 * the library.  1 <= n_pockets <= 1024, 1 <= n < 2^31.  No workspace.
 */
int dock_merge_pockets(const float *d_scores, int32_t n_pockets, int64_t n, float *d_best, int32_t *d_pocket,
                       void *stream);

/*
 * Paper §2: the geometric docking score of one pose, evaluated from scratch
 * (tests and rescoring use it to check the search's incremental scores).
 * Scores explicit poses from scratch (no incremental bookkeeping): pose i is
 * ligand d_lig[i] placed at rigid start d_start[i], then torsion k (sweep
 * order) turned by step d_steps[i][k] for k < B.  d_steps is [n_poses][16].
 * Ligands whose status is not OK score +inf; a descriptor whose ligand or
 * start index is out of range scores NaN.
 */
int dock_score_poses(const dock_grid_desc *g, const float *d_grids, const void *d_pack, int32_t n_lig,
                     int64_t n_atoms_total, const dock_search *s, const int32_t *d_lig, const int32_t *d_start,
                     const uint16_t *d_steps, int64_t n_poses, float *d_scores, void *stream);

/* Static text for a DOCK_* status code. */
const char *dock_error_string(int code);

/* Detail of the last failing call on this thread ("" if none). */
const char *dock_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LIGATE_DOCK_H */
