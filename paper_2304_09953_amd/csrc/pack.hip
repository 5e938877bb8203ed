// Ligand packer: one wavefront per ligand validates the bond tree and derives, with 128-bit
// atom masks held in LDS, the rigid fragments, the core, each torsion's moving set and the
// sweep order, plus per-atom exclusion masks for the clash term; coordinates are centred
// on the unweighted centroid (FP64 sum) and written as SoA.
#include "common.h"

namespace ligate {

struct Mask {
    uint32_t w[4];
};

__device__ __forceinline__ Mask mask_zero() { return Mask{{0u, 0u, 0u, 0u}}; }

__device__ __forceinline__ Mask mask_first(int n) {  // bits 0..n-1
    Mask m;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int lo = 32 * q;
        m.w[q] = n >= lo + 32 ? 0xffffffffu : (n <= lo ? 0u : ((1u << (n - lo)) - 1u));
    }
    return m;
}

__device__ __forceinline__ bool mbit(const Mask &m, int i) { return (m.w[i >> 5] >> (i & 31)) & 1u; }
__device__ __forceinline__ void mset(Mask &m, int i) { m.w[i >> 5] |= 1u << (i & 31); }
__device__ __forceinline__ void mclr(Mask &m, int i) { m.w[i >> 5] &= ~(1u << (i & 31)); }
__device__ __forceinline__ bool mempty(const Mask &m) { return (m.w[0] | m.w[1] | m.w[2] | m.w[3]) == 0u; }
__device__ __forceinline__ int mcount(const Mask &m) {
    return __popc(m.w[0]) + __popc(m.w[1]) + __popc(m.w[2]) + __popc(m.w[3]);
}
__device__ __forceinline__ int mlowest(const Mask &m) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (m.w[q]) return 32 * q + __ffs(m.w[q]) - 1;
    return -1;
}

struct PackShared {
    uint32_t adj[DOCK_MAX_ATOMS][4];   // all bonds
    uint32_t adjn[DOCK_MAX_ATOMS][4];  // non-rotatable bonds only
    int deg[DOCK_MAX_ATOMS];
    int rb_u[DOCK_MAX_TORSIONS], rb_v[DOCK_MAX_TORSIONS];
    int ta[DOCK_MAX_TORSIONS], tb[DOCK_MAX_TORSIONS], tm[DOCK_MAX_TORSIONS];
    uint32_t tmask[DOCK_MAX_TORSIONS][4];
};

// Atoms reachable from `start` over the adjacency in LDS, not using the edge (bu, bv).
__device__ Mask reach(const uint32_t (*adj)[4], int n, int start, int bu, int bv) {
    Mask vis = mask_zero(), fr = mask_zero();
    mset(vis, start);
    mset(fr, start);
    const int lane = lane_id();
    while (!mempty(fr)) {
        uint32_t acc[4] = {0u, 0u, 0u, 0u};
        for (int h = 0; h < 2; ++h) {
            const int i = lane + 64 * h;
            if (i < n && mbit(fr, i)) {
                Mask m;
#pragma unroll
                for (int q = 0; q < 4; ++q) m.w[q] = adj[i][q];
                if (i == bu) mclr(m, bv);
                if (i == bv) mclr(m, bu);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] |= m.w[q];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t nxt = wave_or(acc[q]) & ~vis.w[q];
            fr.w[q] = nxt;
            vis.w[q] |= nxt;
        }
    }
    return vis;
}

struct PackOut {
    LigDesc *desc;
    float *x, *y, *z;
    uint8_t *type;
    uint4 *excl;
    TorRec *tor;
};

__global__ __launch_bounds__(64) void k_pack(const int32_t *__restrict__ atom_off, const float *__restrict__ xyz,
                                             const uint8_t *__restrict__ type, const int32_t *__restrict__ bond_off,
                                             const int32_t *__restrict__ bonds, const uint8_t *__restrict__ rot,
                                             int32_t n_types, int64_t n_atoms_total, PackOut out,
                                             int32_t *__restrict__ status_out) {
    __shared__ PackShared S;
    const int l = blockIdx.x;
    const int lane = lane_id();
    const int a0 = atom_off[l], n = atom_off[l + 1] - a0;
    const int b0 = bond_off[l], nb = bond_off[l + 1] - b0;
    int status = DOCK_LIG_OK;

    // the atom range must also lie inside the packed arrays, which are sized by n_atoms_total
    if (n < 1 || n > DOCK_MAX_ATOMS || a0 < 0 || (int64_t)a0 + n > n_atoms_total) status = DOCK_LIG_NATOMS;
    if (status == DOCK_LIG_OK) {
        bool bad = false;
        for (int i = lane; i < n; i += kWave) bad |= type[a0 + i] >= n_types;
        if (__ballot(bad)) status = DOCK_LIG_TYPE;
    }
    if (status == DOCK_LIG_OK && nb != n - 1) status = DOCK_LIG_NBONDS;
    if (status == DOCK_LIG_OK) {
        bool bad = false;
        for (int e = lane; e < nb; e += kWave) {
            const int u = bonds[2 * (b0 + e)], v = bonds[2 * (b0 + e) + 1];
            bad |= u < 0 || u >= n || v < 0 || v >= n || u == v;
        }
        if (__ballot(bad)) status = DOCK_LIG_BOND_INDEX;
    }
    if (status == DOCK_LIG_OK) {
        for (int i = lane; i < n; i += kWave) {
            S.deg[i] = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) S.adj[i][q] = S.adjn[i][q] = 0u;
        }
        wave_sync();
        for (int e = lane; e < nb; e += kWave) {
            const int u = bonds[2 * (b0 + e)], v = bonds[2 * (b0 + e) + 1];
            atomicAdd(&S.deg[u], 1);
            atomicAdd(&S.deg[v], 1);
            atomicOr(&S.adj[u][v >> 5], 1u << (v & 31));
            atomicOr(&S.adj[v][u >> 5], 1u << (u & 31));
            if (!rot[b0 + e]) {
                atomicOr(&S.adjn[u][v >> 5], 1u << (v & 31));
                atomicOr(&S.adjn[v][u >> 5], 1u << (u & 31));
            }
        }
        wave_sync();
        bool bad = false;
        for (int i = lane; i < n; i += kWave) bad |= S.deg[i] > 4;
        if (__ballot(bad)) status = DOCK_LIG_DEGREE;
    }
    const Mask all = mask_first(n > 0 && n <= DOCK_MAX_ATOMS ? n : 0);
    if (status == DOCK_LIG_OK) {
        const Mask r = reach(S.adj, n, 0, -1, -1);
        if (mcount(r) != n) status = DOCK_LIG_NOT_TREE;
    }
    int B = 0;
    if (status == DOCK_LIG_OK) {
        bool bad = false;
        for (int base = 0; base < nb; base += kWave) {
            const int e = base + lane;
            bool r = false;
            int u = 0, v = 0;
            if (e < nb) {
                r = rot[b0 + e] != 0;
                u = bonds[2 * (b0 + e)];
                v = bonds[2 * (b0 + e) + 1];
                bad |= r && (S.deg[u] < 2 || S.deg[v] < 2);
            }
            const uint64_t bal = __ballot(r);
            const int slot = B + lanes_below(bal);
            if (r && slot < DOCK_MAX_TORSIONS) {
                S.rb_u[slot] = u;
                S.rb_v[slot] = v;
            }
            B += __popcll(bal);
        }
        if (__ballot(bad)) status = DOCK_LIG_TERMINAL_ROT;
        else if (B > DOCK_MAX_TORSIONS) status = DOCK_LIG_NTORSIONS;
    }
    wave_sync();

    if (status != DOCK_LIG_OK) {
        if (lane == 0) {
            out.desc[l] = LigDesc{a0, n, 0, status, 0, 0, 0, 0};
            status_out[l] = status;
        }
        return;
    }

    // centred reference conformer, SoA
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int i = lane; i < n; i += kWave) {
        sx += xyz[3 * (a0 + i) + 0];
        sy += xyz[3 * (a0 + i) + 1];
        sz += xyz[3 * (a0 + i) + 2];
    }
    sx = wave_sum_d(sx) / n;
    sy = wave_sum_d(sy) / n;
    sz = wave_sum_d(sz) / n;
    for (int i = lane; i < n; i += kWave) {
        out.x[a0 + i] = (float)((double)xyz[3 * (a0 + i) + 0] - sx);
        out.y[a0 + i] = (float)((double)xyz[3 * (a0 + i) + 1] - sy);
        out.z[a0 + i] = (float)((double)xyz[3 * (a0 + i) + 2] - sz);
        out.type[a0 + i] = type[a0 + i];
    }

    // rigid fragments in order of their lowest atom; the first largest one is the core
    Mask rem = all, core = mask_zero();
    int best = 0;
    while (!mempty(rem)) {
        const int s = mlowest(rem);
        const Mask comp = reach(S.adjn, n, s, -1, -1);
        const int size = mcount(comp);
        if (size > best) {
            best = size;
            core = comp;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) rem.w[q] &= ~comp.w[q];
    }

    // torsions oriented away from the core
    int sum_m = 0;
    for (int k = 0; k < B; ++k) {
        const int u = S.rb_u[k], v = S.rb_v[k];
        const Mask side_v = reach(S.adj, n, v, u, v);
        bool core_on_v = false;
#pragma unroll
        for (int q = 0; q < 4; ++q) core_on_v |= (side_v.w[q] & core.w[q]) != 0u;
        Mask mv;
#pragma unroll
        for (int q = 0; q < 4; ++q) mv.w[q] = core_on_v ? (all.w[q] & ~side_v.w[q]) : side_v.w[q];
        const int m = mcount(mv);
        sum_m += m;
        if (lane == 0) {
            S.ta[k] = core_on_v ? v : u;
            S.tb[k] = core_on_v ? u : v;
            S.tm[k] = m;
#pragma unroll
            for (int q = 0; q < 4; ++q) S.tmask[k][q] = mv.w[q];
        }
    }
    wave_sync();
    // sweep order: larger moving sets first, ties by input bond order
    if (lane < B) {
        const int mk = S.tm[lane];
        int rank = 0;
        for (int j = 0; j < B; ++j) rank += (S.tm[j] > mk) || (S.tm[j] == mk && j < lane);
        TorRec r;
#pragma unroll
        for (int q = 0; q < 4; ++q) r.mask[q] = S.tmask[lane][q];
        r.a = (uint8_t)S.ta[lane];
        r.b = (uint8_t)S.tb[lane];
        r.m = (uint16_t)mk;
        out.tor[(size_t)l * DOCK_MAX_TORSIONS + rank] = r;
    }

    // per atom: atoms fewer than three bonds away; count the clash pairs
    int pairs = 0;
    for (int i = lane; i < n; i += kWave) {
        Mask e = mask_zero();
        mset(e, i);
        Mask nb1;
#pragma unroll
        for (int q = 0; q < 4; ++q) nb1.w[q] = S.adj[i][q];
#pragma unroll
        for (int q = 0; q < 4; ++q) e.w[q] |= nb1.w[q];
        for (int j = 0; j < n; ++j)
            if (mbit(nb1, j)) {
#pragma unroll
                for (int q = 0; q < 4; ++q) e.w[q] |= S.adj[j][q];
            }
        out.excl[a0 + i] = make_uint4(e.w[0], e.w[1], e.w[2], e.w[3]);
        Mask above = all;  // partners j > i that are not excluded
        for (int j = 0; j <= i; ++j) mclr(above, j);
#pragma unroll
        for (int q = 0; q < 4; ++q) above.w[q] &= ~e.w[q];
        pairs += mcount(above);
    }
    pairs = wave_sum_i(pairs);
    if (lane == 0) {
        out.desc[l] = LigDesc{a0, n, B, DOCK_LIG_OK, sum_m, pairs, 0, 0};
        status_out[l] = DOCK_LIG_OK;
    }
}

}  // namespace ligate

using namespace ligate;

extern "C" int dock_pack_ligands(const int32_t *d_atom_off, const float *d_xyz, const uint8_t *d_type,
                                 const int32_t *d_bond_off, const int32_t *d_bonds, const uint8_t *d_rot,
                                 int32_t n_lig, int64_t n_atoms_total, int32_t n_types, void *d_pack,
                                 size_t *pack_bytes, int32_t *d_status, void *stream) {
    LIGATE_ABI_RANGE();
    LIGATE_REQUIRE(n_lig >= 0 && n_atoms_total >= 0 && n_atoms_total < (1ll << 31), DOCK_ERR_INVALID_ARG,
                   "bad library size (n_lig %d, n_atoms %lld)", n_lig, (long long)n_atoms_total);
    LIGATE_REQUIRE(n_types >= 1 && n_types <= DOCK_MAX_TYPES, DOCK_ERR_LIMIT, "n_types must be in [1, 32]");
    LIGATE_REQUIRE(pack_bytes != nullptr, DOCK_ERR_INVALID_ARG, "pack_bytes is NULL");
    const PackLayout L = PackLayout::make(n_lig, n_atoms_total);
    if (d_pack == nullptr) {
        *pack_bytes = L.total;
        return DOCK_OK;
    }
    LIGATE_REQUIRE(*pack_bytes >= L.total, DOCK_ERR_WORKSPACE, "pack buffer has %zu bytes, %zu needed",
                   *pack_bytes, L.total);
    if (n_lig == 0) return DOCK_OK;
    LIGATE_REQUIRE(d_atom_off && d_bond_off && d_status, DOCK_ERR_INVALID_ARG, "NULL array");
    LIGATE_REQUIRE(n_atoms_total == 0 || (d_xyz && d_type), DOCK_ERR_INVALID_ARG, "NULL atom arrays");
    char *b = (char *)d_pack;
    PackOut o;
    o.desc = (LigDesc *)(b + L.desc);
    o.x = (float *)(b + L.x);
    o.y = (float *)(b + L.y);
    o.z = (float *)(b + L.z);
    o.type = (uint8_t *)(b + L.type);
    o.excl = (uint4 *)(b + L.excl);
    o.tor = (TorRec *)(b + L.tor);
    hipLaunchKernelGGL(k_pack, dim3((unsigned)n_lig), dim3(kWave), 0, (hipStream_t)stream, d_atom_off, d_xyz, d_type,
                       d_bond_off, d_bonds, d_rot, n_types, n_atoms_total, o, d_status);
    return check_launch("dock_pack_ligands");
}
