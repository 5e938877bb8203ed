// Receptor grid build: one thread per (atom type, node), FP64 sum over the protein atoms,
// capped, stored in FP32 as [t][z][y][x] (linear layout) or scattered into the four xy4 records
// that hold the node (xy4 layout, bricked record order), whose differences a second pass forms.
#include "common.h"

namespace ligate {

struct TypeTable {
    double R[DOCK_MAX_TYPES], eps[DOCK_MAX_TYPES], q[DOCK_MAX_TYPES];
};

constexpr int kGridBlock = 256;

__global__ __launch_bounds__(kGridBlock) void k_build_grids(int nx, int ny, int nz, int n_types, float ox, float oy,
                                                          float oz, float h, const float *__restrict__ prot,
                                                          const int32_t *__restrict__ ptype, int n_prot,
                                                          TypeTable tt, double cap, double r_min, double ck,
                                                          int layout, float *__restrict__ out) {
    __shared__ double sx[kGridBlock], sy[kGridBlock], sz[kGridBlock];
    __shared__ int st[kGridBlock];
    __shared__ double r0t[DOCK_MAX_TYPES], epst[DOCK_MAX_TYPES], qqt[DOCK_MAX_TYPES];
    const int t = blockIdx.y;
    const int tid = threadIdx.x;
    const int64_t nxyz = (int64_t)nx * ny * nz;
    const int64_t node = (int64_t)blockIdx.x * kGridBlock + tid;
    if (tid < n_types) {
        r0t[tid] = tt.R[t] + tt.R[tid];
        epst[tid] = sqrt(tt.eps[t] * tt.eps[tid]);
        qqt[tid] = ck * tt.q[t] * tt.q[tid];
    }
    const int i = (int)(node % nx), j = (int)((node / nx) % ny), k = (int)(node / ((int64_t)nx * ny));
    const double X = (double)ox + (double)h * i, Y = (double)oy + (double)h * j, Z = (double)oz + (double)h * k;
    double sum = 0.0;
    for (int base = 0; base < n_prot; base += kGridBlock) {
        __syncthreads();
        if (base + tid < n_prot) {
            sx[tid] = prot[3 * (base + tid) + 0];
            sy[tid] = prot[3 * (base + tid) + 1];
            sz[tid] = prot[3 * (base + tid) + 2];
            st[tid] = ptype[base + tid];
        }
        __syncthreads();
        const int cnt = min(kGridBlock, n_prot - base);
        for (int a = 0; a < cnt; ++a) {
            const double dx = X - sx[a], dy = Y - sy[a], dz = Z - sz[a];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double inv = 1.0 / fmax(r, r_min);
            const int tb = st[a];
            const double s = r0t[tb] * inv, s2 = s * s, s6 = s2 * s2 * s2;
            sum += epst[tb] * (s6 * s6 - 2.0 * s6) + qqt[tb] * inv;
        }
    }
    if (node >= nxyz) return;
    const float v = (float)fmin(sum, cap);
    if (layout == DOCK_LAYOUT_LINEAR) {
        out[(int64_t)t * nxyz + node] = v;
        return;
    }
    // record (X, Y, k) holds nodes (X, Y), (X+1, Y), (X, Y+1), (X+1, Y+1) of plane k, indices
    // modulo n: node (i, j) is component 0 of record (i, j), 1 of (i-1, j), 2 of (i, j-1), 3 of
    // (i-1, j-1)
    const Xy4Geom geo = Xy4Geom::of(nx, ny, nz);
    const uint32_t im = i == 0 ? nx - 1 : i - 1, jm = j == 0 ? ny - 1 : j - 1;
    float *base = out + (size_t)t * (geo.type_bytes() / 4);
    base[geo.offset(i, j, k) / 4 + 0] = v;
    base[geo.offset(im, j, k) / 4 + 1] = v;
    base[geo.offset(i, jm, k) / 4 + 2] = v;
    base[geo.offset(im, jm, k) / 4 + 3] = v;
}

// xy4 records of node values (a, b, c, d) = (G00, G10, G01, G11) -> the plane form (a, b - a, c - a,
// (d - c) - (b - a)), rounded in FP32 exactly as the linear layout's lookups form it; the padding
// records of odd dimensions (never read) are set to zero.
__global__ __launch_bounds__(kGridBlock) void k_xy4_diff(float4 *__restrict__ rec, int64_t n, int nx, int ny, int nz) {
    const int64_t i = (int64_t)blockIdx.x * kGridBlock + threadIdx.x;
    if (i >= n) return;
    const Xy4Geom geo = Xy4Geom::of(nx, ny, nz);
    const int64_t r_type = (int64_t)(geo.type_bytes() / 16);
    const uint32_t in_type = (uint32_t)(i % r_type), brick = in_type >> 2, pos = in_type & 3u;
    const uint32_t x = brick % geo.nxp;
    const uint32_t y = 2u * ((brick / geo.nxp) % geo.nby) + (pos & 1u);
    const uint32_t z = 2u * (brick / (geo.nxp * geo.nby)) + (pos >> 1);
    float4 r = rec[i];
    const float dx = r.y - r.x;
    r = make_float4(r.x, dx, r.z - r.x, (r.w - r.z) - dx);
    if (x >= (uint32_t)nx || y >= (uint32_t)ny || z >= (uint32_t)nz) r = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    rec[i] = r;
}

static int check_desc(const dock_grid_desc *g) {
    LIGATE_REQUIRE(g != nullptr, DOCK_ERR_INVALID_ARG, "grid descriptor is NULL");
    LIGATE_REQUIRE(g->nx >= 2 && g->ny >= 2 && g->nz >= 2, DOCK_ERR_INVALID_ARG, "grid dims must be >= 2");
    LIGATE_REQUIRE((int64_t)g->nx * g->ny * g->nz < (1ll << 24), DOCK_ERR_LIMIT, "grid has >= 2^24 nodes");
    LIGATE_REQUIRE(g->n_types >= 1 && g->n_types <= DOCK_MAX_TYPES, DOCK_ERR_LIMIT, "n_types must be in [1, 32]");
    LIGATE_REQUIRE(g->spacing > 0.0f, DOCK_ERR_INVALID_ARG, "spacing must be > 0");
    LIGATE_REQUIRE(g->layout == DOCK_LAYOUT_LINEAR || g->layout == DOCK_LAYOUT_XY4, DOCK_ERR_INVALID_ARG,
                   "unknown grid layout %d", g->layout);
    // one buffer resource addresses all type grids with 31-bit offsets; offsets inside one xy4
    // type grid are formed in FP32, exact below 2^28 for multiples of 16
    LIGATE_REQUIRE(grid_type_bytes(g) * (uint64_t)g->n_types < (1ull << 31), DOCK_ERR_LIMIT,
                   "grids of all types reach 2^31 bytes");
    LIGATE_REQUIRE(grid_type_bytes(g) < (1ull << 28), DOCK_ERR_LIMIT, "one type grid reaches 2^28 bytes");
    if (g->layout == DOCK_LAYOUT_XY4) {
        // the record offsets take 24-bit multiplies by the strides of y and z pairs (64 nxp - 32
        // and 64 nxp nby - 64)
        const Xy4Geom geo = Xy4Geom::of(g->nx, g->ny, g->nz);
        LIGATE_REQUIRE(64ull * geo.nxp * geo.nby <= (1ull << 24), DOCK_ERR_LIMIT,
                       "xy4 layout: (nx rounded up to even) * ceil(ny / 2) exceeds 2^18");
    }
    LIGATE_REQUIRE(g->boundary == DOCK_BOUNDARY_CLAMP || g->boundary == DOCK_BOUNDARY_PERIODIC,
                   DOCK_ERR_INVALID_ARG, "unknown boundary mode %d", g->boundary);
    return DOCK_OK;
}

int grid_desc_check(const dock_grid_desc *g) { return check_desc(g); }

}  // namespace ligate

using namespace ligate;

extern "C" int dock_grid_bytes(const dock_grid_desc *g, size_t *bytes) {
    LIGATE_ABI_RANGE();
    int rc = check_desc(g);
    if (rc) return rc;
    LIGATE_REQUIRE(bytes != nullptr, DOCK_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = (size_t)(grid_type_bytes(g) * (uint64_t)g->n_types);
    return DOCK_OK;
}

extern "C" int dock_build_grids(const dock_grid_desc *g, const float *d_prot_xyz, const int32_t *d_prot_type,
                                int32_t n_prot, const dock_type_param *h_params, const dock_potential *pot,
                                float *d_grids, void *stream) {
    LIGATE_ABI_RANGE();
    int rc = check_desc(g);
    if (rc) return rc;
    LIGATE_REQUIRE(n_prot >= 0, DOCK_ERR_INVALID_ARG, "n_prot < 0");
    LIGATE_REQUIRE(n_prot == 0 || (d_prot_xyz && d_prot_type), DOCK_ERR_INVALID_ARG, "protein arrays are NULL");
    LIGATE_REQUIRE(h_params && pot && d_grids, DOCK_ERR_INVALID_ARG, "NULL argument");
    LIGATE_REQUIRE(pot->r_min > 0.0, DOCK_ERR_INVALID_ARG, "r_min must be > 0");
    TypeTable tt;
    for (int t = 0; t < DOCK_MAX_TYPES; ++t) {
        const dock_type_param p = t < g->n_types ? h_params[t] : dock_type_param{1.0, 0.0, 0.0};
        LIGATE_REQUIRE(p.eps >= 0.0, DOCK_ERR_INVALID_ARG, "eps of type %d is negative", t);
        tt.R[t] = p.R;
        tt.eps[t] = p.eps;
        tt.q[t] = p.q;
    }
    const int64_t nxyz = (int64_t)g->nx * g->ny * g->nz;
    dim3 grid((unsigned)((nxyz + kGridBlock - 1) / kGridBlock), (unsigned)g->n_types);
    hipLaunchKernelGGL(k_build_grids, grid, dim3(kGridBlock), 0, (hipStream_t)stream, g->nx, g->ny, g->nz,
                       g->n_types, g->origin[0], g->origin[1], g->origin[2], g->spacing, d_prot_xyz, d_prot_type,
                       n_prot, tt, pot->cap, pot->r_min, pot->coulomb_k, g->layout, d_grids);
    if (g->layout == DOCK_LAYOUT_XY4) {
        const int64_t n = (int64_t)(grid_type_bytes(g) / 16) * g->n_types;
        hipLaunchKernelGGL(k_xy4_diff, dim3((unsigned)((n + kGridBlock - 1) / kGridBlock)), dim3(kGridBlock), 0,
                           (hipStream_t)stream, reinterpret_cast<float4 *>(d_grids), n, g->nx, g->ny, g->nz);
    }
    return check_launch("dock_build_grids");
}
