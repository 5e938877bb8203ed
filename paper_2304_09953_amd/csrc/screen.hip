// The docking screen: rigid starts, greedy torsion sweeps, best pose per ligand.
//
// Work decomposition.  A work item is (ligand, batch of rigid starts).  Persistent blocks pop
// items from an atomic counter.  Starts are enumerated translation-major (a batch of n_quat
// starts shares one translation) and items run batch-major, each batch over the ligands in
// order of descending estimated cost: at any time the whole chip works around the same
// translation, so the grid region it reads is about one ligand's extent, which keeps more of
// it in the L2 caches.  A block stages the item's ligand in LDS and its wavefronts take the
// item's starts round-robin.  Within a wavefront, lanes are torsion steps: lane L evaluates the
// angles 2 pi (L + 64 j) / S, j < APL, so one sweep of S angles costs ceil(S / 64) angles per
// lane and the argmin is a single wave reduction.  A start's atom coordinates live in a
// per-wavefront LDS copy (atom i read by lane i and i - 64), which keeps the sweep's registers
// for the lookups.
//
// Scoring inside a sweep.  Turning torsion k moves only its moving set M_k, so the step that
// minimises the score also minimises the part that depends on the step: the grid terms of the
// moving atoms plus the clash of (moving, fixed) pairs.  Each moving atom runs on a circle
// x(t) = p + a cos t + b sin t about the axis, so a pair distance is d^2(t) = A + C cos t +
// D sin t; a pair whose closest approach over the whole circle is beyond the clash cut-off
// cannot contribute and is dropped once per sweep.  The pose score is carried along as
// E <- E - var(0) + var(s*), starting from the rigid pose (grid terms + the clash of the
// reference conformer, which rigid motion does not change).
//
// The per-ligand best (score, start) is an atomicMin on packed ordered keys, so ties go to the
// lowest start.  A replay kernel then reruns the winning start with the same code to recover
// its torsion steps; the result is bitwise identical because every reduction inside a start has
// a fixed order.
#include <math.h>

#include <algorithm>
#include <mutex>

#include "common.h"

namespace ligate {

int grid_desc_check(const dock_grid_desc *g);

struct GridC {
    const float *G;
    uint32_t total_bytes;      // all type grids
    uint32_t type_bytes;       // one type grid
    int nx, ny, nz;
    // linear layout: byte strides of y and z, also as floats (offsets inside one type grid are
    // below 2^26 and multiples of 4, so exact in FP32)
    uint32_t row, plane;
    float frow, fplane;
    // xy4 layout: the record offset is 64 x + 16 y + 32 z + ky (y >> 1) + kz (z >> 1), and the
    // z + 1 record sits at 64 x + 16 y + 32 (z + 1) + ky (y >> 1) + kz ((z + 1) >> 1) with
    // (z + 1) >> 1 = z - (z >> 1); ky, kz < 2^24 (checked with the descriptor), so the products
    // take 24-bit multiplies
    Xy4Geom geo;
    uint32_t ky, kz;
    float mx, my, mz;          // n - 1: clamp bound
    float in_lo, in_x, in_y, in_z;  // inside-the-box test: [kEdge, n - 1 - kEdge] per axis
    float cx, cy, cz;          // n - 2: last cell
    float inv_h, ox_h, oy_h, oz_h;  // grid units: u = x / h - o / h
    float w_h2;                // restraint weight in grid units (w_out h^2)
};

struct SearchC {
    const float *__restrict__ quat;
    const float *__restrict__ trans;
    int n_quat, n_trans, S, QT;
    float cut, cut2, cut2_keep, w;  // clash in grid units: cut-off / h, its square, (cut-off / h + margin)^2,
                                    // weight h^2
    float sw, swc;                  // sqrt(w) and sqrt(w) cut
    int top;                        // starts searched per ligand when they are selected (0: all)
    int passes;                     // greedy passes over the torsions (>= 1)
    int restarts, N;                // torsion restarts per rigid start; searched starts (1 + restarts) QT
    const int32_t *__restrict__ init;  // [restarts][16] initial turns
};

// Coordinates inside a start are in grid units (x - origin) / spacing throughout: the map is a
// similarity, so rotations and torsion turns commute with it, lookups need no conversion, and the
// clash is evaluated with the cut-off divided by h and the weight multiplied by h^2.
struct LigLDS {
    float xr[DOCK_MAX_ATOMS], yr[DOCK_MAX_ATOMS], zr[DOCK_MAX_ATOMS];  // centred reference / h
    uint32_t tof[DOCK_MAX_ATOMS];  // byte offset of the atom's type grid
    uint4 excl[DOCK_MAX_ATOMS];
    TorRec tor[DOCK_MAX_TORSIONS];
    int n, B, status, lig;
};

// Circle coefficients of one moving atom for the current sweep (grid units).
struct Coef {
    float px, py, pz, ax, ay, az, bx, by, bz;
    uint32_t tof;  // type grid byte offset; bit 31 set when the whole circle lies inside the box
    float rho, zz;
};
static_assert(sizeof(Coef) == 48, "Coef layout");
constexpr uint32_t kInside = 0x80000000u;
constexpr float kEdge = 1e-3f;  // margin of the inside-the-box test, in grid units

constexpr int kSurvCap = 128;

struct WaveLDS {
    Coef coef[kWave];
    uint8_t atom[kWave];
    uint16_t sidx[kSurvCap];      // surviving pair: moving slot q | fixed atom j << 8
    float4 surv[kSurvCap];        // its distance coefficients (A, C, D)
    float3 pos[DOCK_MAX_ATOMS];   // the start's current coordinates (grid units)
};

// ---------------------------------------------------------------------------------------------
// Grid lookup (trilinear; clamp + restraint or periodic)
// ---------------------------------------------------------------------------------------------

typedef __amdgpu_buffer_rsrc_t rsrc_t;

__device__ __forceinline__ rsrc_t grid_rsrc(const GridC &g) {
    // raw buffer over all type grids; loads outside it return 0 instead of faulting
    return __builtin_amdgcn_make_buffer_rsrc((void *)g.G, 0, (int)g.total_bytes, 0x00020000);
}

__device__ __forceinline__ float2 ld2(rsrc_t rs, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
}

__device__ __forceinline__ float ld1(rsrc_t rs, uint32_t voff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, 0, 0));
}

// Trilinear interpolation from the two z planes of a cell, each given as (G00, dX, dY, dXY) with
// G00 = G(x0, y0), dX = G(x1, y0) - G00, dY = G(x0, y1) - G00 and dXY = (G(x1, y1) - G(x0, y1)) - dX,
// all differences rounded to FP32: a plane is G00 + fx dX + fy (dY + fx dXY), then a lerp along z.
__device__ __forceinline__ float plane(float fx, float fy, const float4 &r) {
    return fmaf(fy, fmaf(fx, r.w, r.z), fmaf(fx, r.y, r.x));
}

__device__ __forceinline__ float trilerp(float fx, float fy, float fz, const float4 &p0, const float4 &p1) {
    const float c0 = plane(fx, fy, p0), c1 = plane(fx, fy, p1);
    return fmaf(fz, c1 - c0, c0);
}

// The plane form of the corners (G00, G10) = a, (G01, G11) = b, rounded exactly as the xy4 grid
// build forms its records, so both layouts interpolate identically.
__device__ __forceinline__ float4 plane_of(float2 a, float2 b) {
    const float dx = a.y - a.x;
    return make_float4(a.x, dx, b.x - a.x, (b.y - b.x) - dx);
}

// v_cvt_flr_i32_f32: floor and conversion in one instruction (exact for the in-box coordinates it
// is used on).
__device__ __forceinline__ uint32_t floor_u32(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return (uint32_t)r;
}

// Cell byte offset and fractions of grid point u.  off2 receives, in the xy4 layout, the byte
// offset of the (x0, y0, z0 + 1) record minus 32 (the loads add the 32 as an immediate).
// INSIDE: the caller guarantees 0 <= u <= n - 1 - margin, where clamping is the identity and the
// restraint vanishes, so both variants give the same value there.
template <bool INSIDE, int LAYOUT>
__device__ __forceinline__ uint32_t cell(const GridC &g, float ux, float uy, float uz, float &fx, float &fy, float &fz,
                                         float &rest, uint32_t &off2) {
    if constexpr (LAYOUT == DOCK_LAYOUT_XY4) {
        uint32_t x, y, z;
        if constexpr (INSIDE) {
            // u >= 0: u - floor(u) is exact, and v_fract_f32 returns it
            x = floor_u32(ux);
            y = floor_u32(uy);
            z = floor_u32(uz);
            fx = __builtin_amdgcn_fractf(ux);
            fy = __builtin_amdgcn_fractf(uy);
            fz = __builtin_amdgcn_fractf(uz);
            rest = 0.0f;
        } else {
            // fmaxf returns the non-NaN operand, so even a NaN coordinate yields an in-range cell
            const float qx = fminf(fmaxf(ux, 0.0f), g.mx), qy = fminf(fmaxf(uy, 0.0f), g.my),
                        qz = fminf(fmaxf(uz, 0.0f), g.mz);
            const float x0 = floorf(fminf(qx, g.cx)), y0 = floorf(fminf(qy, g.cy)), z0 = floorf(fminf(qz, g.cz));
            fx = qx - x0;
            fy = qy - y0;
            fz = qz - z0;
            x = (uint32_t)x0;
            y = (uint32_t)y0;
            z = (uint32_t)z0;
            const float dx = ux - qx, dy = uy - qy, dz = uz - qz;
            rest = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        }
        const uint32_t hy = (y >> 1) & 0x7fffffu, hz = (z >> 1) & 0x7fffffu, hz1 = (z - hz) & 0xffffffu;
        const uint32_t t = __umul24(hy, g.ky) + (x << 6) + (y << 4) + (z << 5);
        off2 = __umul24(hz1, g.kz) + t;
        return __umul24(hz, g.kz) + t;
    } else {
        float qx = ux, qy = uy, qz = uz, x0, y0, z0;
        if constexpr (INSIDE) {
            x0 = floorf(qx);
            y0 = floorf(qy);
            z0 = floorf(qz);
            rest = 0.0f;
        } else {
            qx = fminf(fmaxf(ux, 0.0f), g.mx);
            qy = fminf(fmaxf(uy, 0.0f), g.my);
            qz = fminf(fmaxf(uz, 0.0f), g.mz);
            x0 = floorf(fminf(qx, g.cx));
            y0 = floorf(fminf(qy, g.cy));
            z0 = floorf(fminf(qz, g.cz));
            const float dx = ux - qx, dy = uy - qy, dz = uz - qz;
            rest = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        }
        fx = qx - x0;
        fy = qy - y0;
        fz = qz - z0;
        off2 = 0;
        return (uint32_t)fmaf(z0, g.fplane, fmaf(y0, g.frow, 4.0f * x0));
    }
}

__device__ __forceinline__ float4 ld4(rsrc_t rs, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, 0));
}

// The two z planes of a cell whose base node is at byte offset `off` (+ soff) in plane form:
// xy4 layout, the stored records (the second at off2 + 32); linear layout, one 8-byte load per
// (y, z) row, with the differences formed here.
struct CellVals {
    float4 p0, p1;
};

template <int LAYOUT>
__device__ __forceinline__ CellVals load_cell(const GridC &g, rsrc_t rs, uint32_t off, uint32_t off2, uint32_t soff) {
    CellVals v;
    if constexpr (LAYOUT == DOCK_LAYOUT_XY4) {
        v.p0 = ld4(rs, off, soff);
        v.p1 = ld4(rs, off2 + 32u, soff);
    } else {
        v.p0 = plane_of(ld2(rs, off, soff), ld2(rs, off, soff + g.row));
        v.p1 = plane_of(ld2(rs, off, soff + g.plane), ld2(rs, off, soff + g.plane + g.row));
    }
    return v;
}

// N clamp-mode lookups whose type offsets are wave-uniform (sof, SGPRs); all N cells' loads are
// issued before any is consumed.
template <int N, bool INSIDE, int LAYOUT>
__device__ __forceinline__ void lookup_group(const GridC &g, rsrc_t rs, const uint32_t (&sof)[N], const float (&ux)[N],
                                             const float (&uy)[N], const float (&uz)[N], float (&out)[N]) {
    uint32_t off[N], off2[N];
    float fx[N], fy[N], fz[N], rest[N];
#pragma unroll
    for (int k = 0; k < N; ++k)
        off[k] = cell<INSIDE, LAYOUT>(g, ux[k], uy[k], uz[k], fx[k], fy[k], fz[k], rest[k], off2[k]);
    CellVals cv[N];
#pragma unroll
    for (int k = 0; k < N; ++k) cv[k] = load_cell<LAYOUT>(g, rs, off[k], off2[k], sof[k]);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float v = trilerp(fx[k], fy[k], fz[k], cv[k].p0, cv[k].p1);
        out[k] = INSIDE ? v : fmaf(g.w_h2, rest[k], v);
    }
}

// One lookup whose type offset differs between lanes (rigid placement, pose scoring).
template <int BOUNDARY, int LAYOUT>
__device__ __forceinline__ float lookup_lane(const GridC &g, rsrc_t rs, uint32_t tof, float ux, float uy, float uz) {
    if constexpr (BOUNDARY == DOCK_BOUNDARY_CLAMP) {
        float fx, fy, fz, rest;
        uint32_t off2;
        const uint32_t off = cell<false, LAYOUT>(g, ux, uy, uz, fx, fy, fz, rest, off2) + tof;
        const CellVals v = load_cell<LAYOUT>(g, rs, off, off2 + tof, 0);
        return fmaf(g.w_h2, rest, trilerp(fx, fy, fz, v.p0, v.p1));
    } else if constexpr (LAYOUT == DOCK_LAYOUT_XY4) {
        // records wrap in x and y; the z neighbour is the record of plane jz
        const float fx0 = floorf(ux), fy0 = floorf(uy), fz0 = floorf(uz);
        const float fx = ux - fx0, fy = uy - fy0, fz = uz - fz0;
        int ix = (int)fx0 % g.nx, iy = (int)fy0 % g.ny, iz = (int)fz0 % g.nz;
        ix += ix < 0 ? g.nx : 0;
        iy += iy < 0 ? g.ny : 0;
        iz += iz < 0 ? g.nz : 0;
        const int jz = iz + 1 == g.nz ? 0 : iz + 1;
        return trilerp(fx, fy, fz, ld4(rs, tof + g.geo.offset(ix, iy, iz), 0), ld4(rs, tof + g.geo.offset(ix, iy, jz), 0));
    } else {
        const float fx0 = floorf(ux), fy0 = floorf(uy), fz0 = floorf(uz);
        const float fx = ux - fx0, fy = uy - fy0, fz = uz - fz0;
        int ix = (int)fx0 % g.nx, iy = (int)fy0 % g.ny, iz = (int)fz0 % g.nz;
        ix += ix < 0 ? g.nx : 0;
        iy += iy < 0 ? g.ny : 0;
        iz += iz < 0 ? g.nz : 0;
        const int jx = ix + 1 == g.nx ? 0 : ix + 1, jy = iy + 1 == g.ny ? 0 : iy + 1,
                  jz = iz + 1 == g.nz ? 0 : iz + 1;
        const uint32_t r00 = tof + 4u * (uint32_t)(g.nx * (iy + g.ny * iz));
        const uint32_t r10 = tof + 4u * (uint32_t)(g.nx * (jy + g.ny * iz));
        const uint32_t r01 = tof + 4u * (uint32_t)(g.nx * (iy + g.ny * jz));
        const uint32_t r11 = tof + 4u * (uint32_t)(g.nx * (jy + g.ny * jz));
        const float2 a = make_float2(ld1(rs, r00 + 4 * ix), ld1(rs, r00 + 4 * jx));
        const float2 b = make_float2(ld1(rs, r10 + 4 * ix), ld1(rs, r10 + 4 * jx));
        const float2 c = make_float2(ld1(rs, r01 + 4 * ix), ld1(rs, r01 + 4 * jx));
        const float2 d = make_float2(ld1(rs, r11 + 4 * ix), ld1(rs, r11 + 4 * jx));
        return trilerp(fx, fy, fz, plane_of(a, b), plane_of(c, d));
    }
}

// ---------------------------------------------------------------------------------------------
// Ligand staging and the per-start greedy pass (one wavefront)
// ---------------------------------------------------------------------------------------------

// Cooperative load of ligand `lig` into LDS by `nthreads` threads; the caller syncs.
__device__ void load_ligand(LigLDS &L, const PackView &pk, int lig, const GridC &g, int tid, int nthreads) {
    const LigDesc d = pk.desc[lig];
    if (tid == 0) {
        L.n = d.n;
        L.B = d.B;
        L.status = d.status;
        L.lig = lig;
    }
    if (d.status != DOCK_LIG_OK) return;
    const uint32_t tbytes = g.type_bytes;
    for (int i = tid; i < d.n; i += nthreads) {
        L.xr[i] = pk.x[d.atom_off + i] * g.inv_h;
        L.yr[i] = pk.y[d.atom_off + i] * g.inv_h;
        L.zr[i] = pk.z[d.atom_off + i] * g.inv_h;
        L.tof[i] = (uint32_t)pk.type[d.atom_off + i] * tbytes;
        L.excl[i] = pk.excl[d.atom_off + i];
    }
    for (int k = tid; k < d.B; k += nthreads) L.tor[k] = pk.tor[(size_t)lig * DOCK_MAX_TORSIONS + k];
}

// Clash energy of the reference conformer (pairs three or more bonds apart), summed over the wave.
__device__ float rigid_clash(const LigLDS &L, const SearchC &s) {
    const int lane = lane_id();
    float acc = 0.0f;
    for (int i = 0; i < L.n; ++i) {
        const float xi = L.xr[i], yi = L.yr[i], zi = L.zr[i];
        const uint4 ex = L.excl[i];
        for (int j = i + 1 + lane; j < L.n; j += kWave) {
            if (mask_has(ex, j)) continue;
            const float dx = L.xr[j] - xi, dy = L.yr[j] - yi, dz = L.zr[j] - zi;
            const float d = __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
            const float t = fmaxf(s.cut - d, 0.0f);
            acc = fmaf(s.w * t, t, acc);
        }
    }
    return wave_sum(acc);
}

__device__ __forceinline__ float shfl_f(float v, int src) { return __shfl(v, src); }

// Circle coefficients of the atom at `x` for the axis through `xa` with unit direction `u`.
__device__ __forceinline__ void circle(float ux, float uy, float uz, float xax, float xay, float xaz, float x, float y,
                                       float z, float &px, float &py, float &pz, float &ax, float &ay, float &az,
                                       float &bx, float &by, float &bz) {
    const float vx = x - xax, vy = y - xay, vz = z - xaz;
    const float zz = fmaf(ux, vx, fmaf(uy, vy, uz * vz));
    px = fmaf(zz, ux, xax);
    py = fmaf(zz, uy, xay);
    pz = fmaf(zz, uz, xaz);
    ax = fmaf(-zz, ux, vx);
    ay = fmaf(-zz, uy, vy);
    az = fmaf(-zz, uz, vz);
    bx = uy * vz - uz * vy;
    by = uz * vx - ux * vz;
    bz = ux * vy - uy * vx;
}

// Per-lane cos/sin of the lane's angles 2 pi (lane + 64 j) / S.
template <int APL>
__device__ __forceinline__ void angle_table(int S, float (&cs)[APL], float (&sn)[APL]) {
    const int lane = lane_id();
#pragma unroll
    for (int j = 0; j < APL; ++j) {
        const int st = lane + kWave * j;
        float sv, cv;
        sincospif(2.0f * (float)st / (float)S, &sv, &cv);
        cs[j] = cv;
        sn[j] = sv;
    }
}

// Rigid start p (< QT) in grid units: quaternion rotation of the reference, then the translation.
__device__ __forceinline__ void place(const GridC &g, const SearchC &s, const LigLDS &L, int p, float (&cx)[2],
                                      float (&cy)[2], float (&cz)[2]) {
    const int lane = lane_id();
    const int iq = p / s.n_trans, it = p - iq * s.n_trans;
    float qw = s.quat[4 * iq], qx = s.quat[4 * iq + 1], qy = s.quat[4 * iq + 2], qz = s.quat[4 * iq + 3];
    const float qn = 1.0f / sqrtf(fmaf(qw, qw, fmaf(qx, qx, fmaf(qy, qy, qz * qz))));
    qw *= qn; qx *= qn; qy *= qn; qz *= qn;
    const float r00 = 1.0f - 2.0f * (qy * qy + qz * qz), r01 = 2.0f * (qx * qy - qw * qz), r02 = 2.0f * (qx * qz + qw * qy);
    const float r10 = 2.0f * (qx * qy + qw * qz), r11 = 1.0f - 2.0f * (qx * qx + qz * qz), r12 = 2.0f * (qy * qz - qw * qx);
    const float r20 = 2.0f * (qx * qz - qw * qy), r21 = 2.0f * (qy * qz + qw * qx), r22 = 1.0f - 2.0f * (qx * qx + qy * qy);
    const float tx = fmaf(s.trans[3 * it], g.inv_h, -g.ox_h);
    const float ty = fmaf(s.trans[3 * it + 1], g.inv_h, -g.oy_h);
    const float tz = fmaf(s.trans[3 * it + 2], g.inv_h, -g.oz_h);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = lane + kWave * h;
        cx[h] = cy[h] = cz[h] = 0.0f;
        if (i < L.n) {
            const float x = L.xr[i], y = L.yr[i], z = L.zr[i];
            cx[h] = fmaf(r00, x, fmaf(r01, y, fmaf(r02, z, tx)));
            cy[h] = fmaf(r10, x, fmaf(r11, y, fmaf(r12, z, ty)));
            cz[h] = fmaf(r20, x, fmaf(r21, y, fmaf(r22, z, tz)));
        }
    }
}

// Axis of torsion k from the current coordinates: the a end and the unit direction a -> b.
__device__ __forceinline__ void axis(const TorRec &tr, const float (&cx)[2], const float (&cy)[2], const float (&cz)[2],
                                     float &xax, float &xay, float &xaz, float &ux, float &uy, float &uz) {
    const int a = tr.a, b = tr.b;
    xax = shfl_f(a < kWave ? cx[0] : cx[1], a & 63);
    xay = shfl_f(a < kWave ? cy[0] : cy[1], a & 63);
    xaz = shfl_f(a < kWave ? cz[0] : cz[1], a & 63);
    const float xbx = shfl_f(b < kWave ? cx[0] : cx[1], b & 63);
    const float xby = shfl_f(b < kWave ? cy[0] : cy[1], b & 63);
    const float xbz = shfl_f(b < kWave ? cz[0] : cz[1], b & 63);
    ux = xbx - xax;
    uy = xby - xay;
    uz = xbz - xaz;
    const float un = __builtin_amdgcn_rsqf(fmaf(ux, ux, fmaf(uy, uy, uz * uz)));  // 1 ulp
    ux *= un;
    uy *= un;
    uz *= un;
}

// The same axis from the wave's LDS copy of the coordinates; the values are wave-uniform and are
// moved to scalar registers.
__device__ __forceinline__ float uniform_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ void axis_lds(const TorRec &tr, const WaveLDS &W, float &xax, float &xay, float &xaz,
                                         float &ux, float &uy, float &uz) {
    const float3 xa = W.pos[tr.a], xb = W.pos[tr.b];
    ux = xb.x - xa.x;
    uy = xb.y - xa.y;
    uz = xb.z - xa.z;
    const float un = __builtin_amdgcn_rsqf(fmaf(ux, ux, fmaf(uy, uy, uz * uz)));  // 1 ulp
    xax = uniform_f(xa.x);
    xay = uniform_f(xa.y);
    xaz = uniform_f(xa.z);
    ux = uniform_f(ux * un);
    uy = uniform_f(uy * un);
    uz = uniform_f(uz * un);
}

// Score of the conformer in registers from scratch: every atom's grid term and every clash pair.
template <int BOUNDARY, int LAYOUT>
__device__ float direct_score(const GridC &g, rsrc_t rs, const SearchC &s, const LigLDS &L, const float (&cx)[2],
                              const float (&cy)[2], const float (&cz)[2]) {
    const int lane = lane_id();
    const int n = L.n;
    float acc = 0.0f;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = lane + kWave * h;
        if (i < n) acc += lookup_lane<BOUNDARY, LAYOUT>(g, rs, L.tof[i], cx[h], cy[h], cz[h]);
    }
    for (int i = 0; i < n; ++i) {
        const float xi = __shfl(i < kWave ? cx[0] : cx[1], i & 63);
        const float yi = __shfl(i < kWave ? cy[0] : cy[1], i & 63);
        const float zi = __shfl(i < kWave ? cz[0] : cz[1], i & 63);
        const uint4 ex = L.excl[i];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = lane + kWave * h;
            if (j > i && j < n && !mask_has(ex, j)) {
                const float dx = cx[h] - xi, dy = cy[h] - yi, dz = cz[h] - zi;
                const float d = __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
                const float t = fmaxf(s.cut - d, 0.0f);
                acc = fmaf(s.w * t, t, acc);
            }
        }
    }
    return wave_sum(acc);
}

// Turns torsion k (axis and moving mask given) of the conformer in W.pos by step st of the lane
// angle tables (the angle 2 pi st / S, held by lane st mod 64 in group st / 64).
template <int APL>
__device__ __forceinline__ void turn_torsion(WaveLDS &W, int n, const uint4 &mask, float xax, float xay, float xaz,
                                             float ux, float uy, float uz, int st, const float (&cs)[APL],
                                             const float (&sn)[APL]) {
    const int lane = lane_id();
    const int jb = st / kWave, owner = st - jb * kWave;
    float csel = cs[0], ssel = sn[0];
#pragma unroll
    for (int j = 1; j < APL; ++j)
        if (j == jb) {
            csel = cs[j];
            ssel = sn[j];
        }
    const float cb = __shfl(csel, owner), sb = __shfl(ssel, owner);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = lane + kWave * h;
        if (i < n && mask_has(mask, i)) {
            const float3 x = W.pos[i];
            float px, py, pz, ax, ay, az, bx, by, bz;
            circle(ux, uy, uz, xax, xay, xaz, x.x, x.y, x.z, px, py, pz, ax, ay, az, bx, by, bz);
            W.pos[i] = make_float3(fmaf(ax, cb, fmaf(bx, sb, px)), fmaf(ay, cb, fmaf(by, sb, py)),
                                   fmaf(az, cb, fmaf(bz, sb, pz)));
        }
    }
    wave_sync();
}

// The conformer in W.pos scored from scratch (every atom's grid term and every clash pair).
template <int BOUNDARY, int LAYOUT>
__device__ float direct_score_lds(const GridC &g, rsrc_t rs, const SearchC &s, const LigLDS &L, const WaveLDS &W) {
    const int lane = lane_id(), n = L.n;
    float cx[2], cy[2], cz[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = lane + kWave * h;
        const float3 x = i < n ? W.pos[i] : make_float3(0.0f, 0.0f, 0.0f);
        cx[h] = x.x;
        cy[h] = x.y;
        cz[h] = x.z;
    }
    return direct_score<BOUNDARY, LAYOUT>(g, rs, s, L, cx, cy, cz);
}

// The greedy passes from searched start e (rigid start e mod QT; for restart r = e / QT >= 1,
// each torsion first turned by its initial step).  Returns the final score (identical on all lanes);
// lane k (< B) receives torsion k's total turn (initial turn and the passes, modulo S) in
// `my_step`.  The start's coordinates live in the wave's LDS copy W.pos (atom i at W.pos[i]), not
// in registers, so that the lookups of a sweep run with fewer live registers.
template <int APL, int BOUNDARY, int LAYOUT>
__device__ float run_start(const GridC &g, rsrc_t rs, const SearchC &s, const LigLDS &L, WaveLDS &W, int e,
                           float clash_ref, const float (&cs)[APL], const float (&sn)[APL], int &my_step) {
    const int lane = lane_id();
    const int n = L.n;
    const int restart = s.restarts ? e / s.QT : 0, p = e - restart * s.QT;
    float eg = 0.0f;
    {
        float cx[2], cy[2], cz[2];
        place(g, s, L, p, cx, cy, cz);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = lane + kWave * h;
            if (i < n) {
                eg += lookup_lane<BOUNDARY, LAYOUT>(g, rs, L.tof[i], cx[h], cy[h], cz[h]);
                W.pos[i] = make_float3(cx[h], cy[h], cz[h]);
            }
        }
    }
    wave_sync();
    float E = wave_sum(eg) + clash_ref;
    my_step = 0;
    if (restart > 0) {  // the restart's initial turns (a zero turn leaves the torsion as it is)
        bool turned = false;
        for (int k = 0; k < L.B; ++k) {
            const int st = ((s.init[(restart - 1) * DOCK_MAX_TORSIONS + k] % s.S) + s.S) % s.S;
            if (lane == k) my_step = st;
            if (st == 0) continue;
            turned = true;
            const TorRec tr = L.tor[k];
            float xax, xay, xaz, ux, uy, uz;
            axis_lds(tr, W, xax, xay, xaz, ux, uy, uz);
            turn_torsion<APL>(W, n, mask_without(make_uint4(tr.mask[0], tr.mask[1], tr.mask[2], tr.mask[3]), tr.b),
                              xax, xay, xaz,
                              ux, uy, uz, st, cs, sn);
        }
        if (turned) E = direct_score_lds<BOUNDARY, LAYOUT>(g, rs, s, L, W);
    }
    // The score is carried incrementally in FP32; when it passed through values much larger than
    // the final one (atoms far outside the box or clashing in the rigid pose), the cancellation
    // would cost accuracy, so the final conformer is then rescored from scratch.
    float Emax = fabsf(E);

    // lookups are grouped four at a time: NJ angles of NA moving atoms
    constexpr int NJ = APL < 4 ? APL : 4;
    constexpr int NA = 4 / NJ;

    // the sweeps of all passes: torsion k runs 0..B-1 in every pass
    for (int sweep = 0, k = 0; sweep < s.passes * L.B; ++sweep, k = k + 1 == L.B ? 0 : k + 1) {
        const TorRec tr = L.tor[k];
        // the moving side; its atom b lies on the axis, so its position, its grid term and its distances
        // to every other atom stay the same through the sweep: only the other moving atoms are turned
        // and scored, and b is neither moving nor fixed for the clash pairs
        const uint4 mask = make_uint4(tr.mask[0], tr.mask[1], tr.mask[2], tr.mask[3]);
        const uint4 turn = mask_without(mask, tr.b);
        float xax, xay, xaz, ux, uy, uz;
        axis_lds(tr, W, xax, xay, xaz, ux, uy, uz);

        // angles past S start at +inf, so they never win the argmin
        float e[APL];
#pragma unroll
        for (int j = 0; j < APL; ++j) e[j] = lane + kWave * j < s.S ? 0.0f : INFINITY;
        int nsurv = 0, nbuilt = 0;

        // distance coefficients of the survivors [nbuilt, nsurv), whose moving slots refer to
        // the coefficients currently in W.coef: d^2(t) = A + C cos t + D sin t
        auto build = [&]() {
            for (int i = nbuilt + lane; i < nsurv; i += kWave) {
                const uint32_t id = W.sidx[i];
                const Coef c = W.coef[id & 0xffu];
                const float3 xj = W.pos[id >> 8];
                const float wx = c.px - xj.x, wy = c.py - xj.y, wz = c.pz - xj.z;
                const float A = fmaf(wx, wx, fmaf(wy, wy, fmaf(wz, wz, c.rho * c.rho)));
                const float C = 2.0f * fmaf(wx, c.ax, fmaf(wy, c.ay, wz * c.az));
                const float D = 2.0f * fmaf(wx, c.bx, fmaf(wy, c.by, wz * c.bz));
                W.surv[i] = make_float4(A, C, D, 0.0f);
            }
            nbuilt = nsurv;
        };

        // A kept pair clashes only on part of its circle: the penalty of an angle group is
        // evaluated only when some lane of the wavefront is inside the cut-off there.
        // The penalty w (c - d)^2 is accumulated as t^2 with t = max(sqrt(w) c - sqrt(w) d, 0); d^2 that
        // rounding made slightly negative (coincident atoms) is taken by magnitude.
        auto flush = [&](int cnt) {
            for (int q = 0; q < cnt; ++q) {
                const float4 acd = W.surv[q];
#pragma unroll
                for (int j = 0; j < APL; ++j) {
                    const float d2 = fmaf(acd.y, cs[j], fmaf(acd.z, sn[j], acd.x));
                    if (__ballot(d2 < s.cut2)) {
                        const float t = fmaxf(fmaf(-s.sw, __builtin_amdgcn_sqrtf(fabsf(d2)), s.swc), 0.0f);
                        e[j] = fmaf(t, t, e[j]);
                    }
                }
            }
        };

#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (kWave * h >= n) break;
            const int i = lane + kWave * h;
            const bool mv = i < n && mask_has_lane(turn, h, lane);
            const uint64_t bal = __ballot(mv);
            const int cnt = __popcll(bal);
            if (mv) {
                const float3 x = W.pos[i];
                Coef c;
                circle(ux, uy, uz, xax, xay, xaz, x.x, x.y, x.z, c.px, c.py, c.pz, c.ax, c.ay, c.az, c.bx, c.by, c.bz);
                c.rho = __builtin_amdgcn_sqrtf(fmaf(c.ax, c.ax, fmaf(c.ay, c.ay, c.az * c.az)));
                c.zz = fmaf(ux, x.x - xax, fmaf(uy, x.y - xay, uz * (x.z - xaz)));
                const bool inside = c.px - c.rho >= g.in_lo && c.py - c.rho >= g.in_lo && c.pz - c.rho >= g.in_lo &&
                                    c.px + c.rho <= g.in_x && c.py + c.rho <= g.in_y && c.pz + c.rho <= g.in_z;
                c.tof = L.tof[i] | (inside ? kInside : 0u);
                const int slot = lanes_below(bal);
                W.coef[slot] = c;
                W.atom[slot] = (uint8_t)i;
            }
            wave_sync();
            // grid terms of the moving atoms on their circles
            for (int q0 = 0; q0 < cnt; q0 += NA) {
                Coef c[NA];
                uint32_t sof[NA];
                bool all_inside = true;
#pragma unroll
                for (int a = 0; a < NA; ++a) {
                    c[a] = W.coef[min(q0 + a, cnt - 1)];
                    const uint32_t t = (uint32_t)__builtin_amdgcn_readfirstlane((int)c[a].tof);
                    sof[a] = t & ~kInside;
                    all_inside = all_inside && (t & kInside);
                }
#pragma unroll
                for (int j0 = 0; j0 < APL; j0 += NJ) {
                    float gx[4], gy[4], gz[4], v[4];
                    uint32_t so[4];
#pragma unroll
                    for (int a = 0; a < NA; ++a)
#pragma unroll
                        for (int jj = 0; jj < NJ; ++jj) {
                            const int idx = a * NJ + jj, j = j0 + jj;
                            gx[idx] = fmaf(c[a].ax, cs[j], fmaf(c[a].bx, sn[j], c[a].px));
                            gy[idx] = fmaf(c[a].ay, cs[j], fmaf(c[a].by, sn[j], c[a].py));
                            gz[idx] = fmaf(c[a].az, cs[j], fmaf(c[a].bz, sn[j], c[a].pz));
                            so[idx] = sof[a];
                        }
                    if constexpr (BOUNDARY == DOCK_BOUNDARY_CLAMP) {
                        if (all_inside) {
                            lookup_group<4, true, LAYOUT>(g, rs, so, gx, gy, gz, v);
                        } else {  // the clamp path needs more registers: two groups of two
#pragma unroll
                            for (int hh = 0; hh < 4; hh += 2) {
                                const uint32_t so2[2] = {so[hh], so[hh + 1]};
                                const float gx2[2] = {gx[hh], gx[hh + 1]}, gy2[2] = {gy[hh], gy[hh + 1]},
                                            gz2[2] = {gz[hh], gz[hh + 1]};
                                float v2[2];
                                lookup_group<2, false, LAYOUT>(g, rs, so2, gx2, gy2, gz2, v2);
                                v[hh] = v2[0];
                                v[hh + 1] = v2[1];
                            }
                        }
                    } else {
#pragma unroll
                        for (int idx = 0; idx < 4; ++idx) v[idx] = lookup_lane<BOUNDARY, LAYOUT>(g, rs, so[idx], gx[idx], gy[idx], gz[idx]);
                    }
#pragma unroll
                    for (int a = 0; a < NA; ++a)
                        if (q0 + a < cnt)
#pragma unroll
                            for (int jj = 0; jj < NJ; ++jj) e[j0 + jj] += v[a * NJ + jj];
                }
            }
            // fixed atoms: cylinder coordinates about the axis (radius +inf for the others, so that
            // no pair with them passes the closest-approach test)
            float zj[2], rj[2];
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const int jj = lane + kWave * h2;
                zj[h2] = 0.0f;
                rj[h2] = INFINITY;
                if (jj < n && !mask_has_lane(mask, h2, lane)) {
                    const float3 x = W.pos[jj];
                    const float vx = x.x - xax, vy = x.y - xay, vz = x.z - xaz;
                    zj[h2] = fmaf(ux, vx, fmaf(uy, vy, uz * vz));
                    const float ox = fmaf(-zj[h2], ux, vx), oy = fmaf(-zj[h2], uy, vy), oz = fmaf(-zj[h2], uz, vz);
                    rj[h2] = __builtin_amdgcn_sqrtf(fmaf(ox, ox, fmaf(oy, oy, oz * oz)));
                }
            }
            // (moving, fixed) clash pairs that can come within the cut-off somewhere on the circle
            for (int q = 0; q < cnt; ++q) {
                const float rho = W.coef[q].rho, zq = W.coef[q].zz;
                const uint4 ex = L.excl[W.atom[q]];
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2) {
                    if (kWave * h2 >= n) break;
                    const int jj = lane + kWave * h2;
                    const float dr = rho - rj[h2], dz = zq - zj[h2];
                    const bool keep = fmaf(dr, dr, dz * dz) < s.cut2_keep && !mask_has_lane(ex, h2, lane);
                    const uint64_t kb = __ballot(keep);
                    if (keep) W.sidx[nsurv + lanes_below(kb)] = (uint16_t)(q | (jj << 8));
                    nsurv += __popcll(kb);
                    if (nsurv >= kWave) {
                        wave_sync();
                        build();
                        wave_sync();
                        flush(nsurv);
                        nsurv = nbuilt = 0;
                        wave_sync();
                    }
                }
            }
            // the next half overwrites W.coef: form the pending survivors' coefficients now
            wave_sync();
            build();
            wave_sync();
        }
        if (nsurv) {
            wave_sync();
            flush(nsurv);
            wave_sync();
        }

        // argmin over the S steps, ties to the lowest step: the wave minimum, then the first step
        // (angle group j, then lane) that attains it
        float emin = e[0];
#pragma unroll
        for (int j = 1; j < APL; ++j) emin = min_nonan(emin, e[j]);
        const float ebest = wave_min(emin);
        int sbest = 0;
#pragma unroll
        for (int j = APL - 1; j >= 0; --j) {
            const uint64_t hit = __ballot(e[j] == ebest);
            if (hit) sbest = kWave * j + (int)__builtin_ctzll(hit);
        }
        const float e0 = __shfl(e[0], 0);
        E += ebest - e0;
        Emax = fmaxf(Emax, fabsf(E));

        // apply the winning step
        turn_torsion<APL>(W, n, turn, xax, xay, xaz, ux, uy, uz, sbest, cs, sn);
        if (lane == k) {  // total turn of torsion k over the passes, modulo S
            my_step += sbest;
            my_step -= my_step >= s.S ? s.S : 0;
        }
    }
    if (Emax > 16.0f * fmaxf(1.0f, fabsf(E))) E = direct_score_lds<BOUNDARY, LAYOUT>(g, rs, s, L, W);
    return E;
}

// The pose (searched start e, total turns steps[k] of torsion k in sweep order) in registers, grid
// units: rigid start e mod QT, then each torsion turned once by its total.  The angles are formed
// here with sincospif (dock_score_poses and the rescoring path share this code, so they build the
// same conformers).
__device__ __forceinline__ void build_pose(const GridC &g, const SearchC &s, const LigLDS &L, int e,
                                           const uint16_t *steps, float (&cx)[2], float (&cy)[2], float (&cz)[2]) {
    const int lane = lane_id(), n = L.n;
    place(g, s, L, e % s.QT, cx, cy, cz);
    for (int k = 0; k < L.B; ++k) {
        const TorRec tr = L.tor[k];
        // the moving side without its axis atom b, which a turn leaves where it is (as in the sweeps)
        const uint4 mask = mask_without(make_uint4(tr.mask[0], tr.mask[1], tr.mask[2], tr.mask[3]), tr.b);
        float xax, xay, xaz, ux, uy, uz;
        axis(tr, cx, cy, cz, xax, xay, xaz, ux, uy, uz);
        float sb, cb;
        sincospif(2.0f * (float)steps[k] / (float)s.S, &sb, &cb);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = lane + kWave * h;
            if (i < n && mask_has(mask, i)) {
                float px, py, pz, ax, ay, az, bx, by, bz;
                circle(ux, uy, uz, xax, xay, xaz, cx[h], cy[h], cz[h], px, py, pz, ax, ay, az, bx, by, bz);
                cx[h] = fmaf(ax, cb, fmaf(bx, sb, px));
                cy[h] = fmaf(ay, cb, fmaf(by, sb, py));
                cz[h] = fmaf(az, cb, fmaf(bz, sb, pz));
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------------------------

struct ScreenArgs {
    GridC g;
    SearchC s;
    PackView pk;
    const uint64_t *order;   // cost-sorted keys, ligand index in the low 32 bits
    uint64_t *best_key;      // [n_lig]
    unsigned long long *counter;  // 64-bit: n_items plus one exit pop per block may pass 2^31
    float *start_scores;     // optional [n_lig][N]
    uint16_t *start_steps;   // optional [n_lig][QT][16]
    const uint32_t *sel;     // [n_lig][s.top] starts to search when s.top > 0
    int n_lig, P, bpl, nw;
    int64_t n_items;
};

__global__ void k_screen_init(uint64_t *best_key, int n_lig, unsigned long long *counter, uint64_t *pose_count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_lig) best_key[i] = ~0ull;
    if (i == 0) {
        *counter = 0ull;
        if (pose_count) *pose_count = 0ull;
    }
}

// Planner: cost-descending order (ties by ligand index); invalid ligands last.  Poses: every
// rigid start once, plus (S - 1) new poses per torsion sweep of each searched start.
// n_first: poses scored before the sweeps (every rigid start when starts are selected, otherwise
// every searched start's first conformer).
__global__ void k_screen_plan(const LigDesc *desc, int n_lig, int S, uint64_t *keys, uint64_t *pose_count,
                              int n_first, int n_searched, int passes) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t poses = 0;
    if (l < n_lig) {
        const LigDesc d = desc[l];
        uint64_t cost = 0;
        if (d.status == DOCK_LIG_OK) {
            cost = (uint64_t)d.n + (uint64_t)passes * ((uint64_t)(S - 1) * (uint64_t)d.sum_m + (uint64_t)d.n_pairs);
            poses = (uint64_t)n_first + (uint64_t)n_searched * (uint64_t)passes * (uint64_t)d.B * (uint64_t)(S - 1);
        }
        if (cost > 0xffffffffull) cost = 0xffffffffull;
        keys[l] = ((uint64_t)(~(uint32_t)cost) << 32) | (uint32_t)l;
    }
    if (pose_count) {
        // per-wave partial sums, one atomic per wave
        uint32_t lo = (uint32_t)poses, hi = (uint32_t)(poses >> 32);
        uint64_t tot = 0;
        for (int src = 0; src < kWave; ++src)
            tot += ((uint64_t)(uint32_t)__shfl((int)hi, src) << 32) | (uint32_t)__shfl((int)lo, src);
        if (lane_id() == 0 && tot) atomicAdd((unsigned long long *)pose_count, (unsigned long long)tot);
    }
}

constexpr int kTopBlock = 256;

// Exclusive prefix sum over the kTopBlock threads of a block (thread order); `scratch` holds one
// value per wavefront.  All threads must call it.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *scratch) {
    const int lane = lane_id(), w = threadIdx.x / kWave;
    uint32_t inc = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)inc, off);
        if (lane >= off) inc += o;
    }
    if (lane == kWave - 1) scratch[w] = inc;
    __syncthreads();
    uint32_t base = 0;
    for (int q = 0; q < w; ++q) base += scratch[q];
    __syncthreads();
    return base + inc - v;
}

struct SelectScratch {
    uint32_t hist[256];
    uint32_t scan[2][kTopBlock / kWave];
    uint32_t prefix, need;
};

// The K lowest of the n keys key[0..n) (in LDS), ties to the lower index, found by a radix select
// eight bits at a time from the top; their indices are written to out[0..K) in increasing order.
// 1 <= K <= n.  All kTopBlock threads of the block must call it.
__device__ void block_select_lowest(const uint32_t *key, int n, int K, uint32_t *out, SelectScratch &sc) {
    const int tid = threadIdx.x;
    // the K-th smallest key; `need` of the keys equal to it belong to the K lowest
    uint32_t prefix = 0, mask = 0, need = (uint32_t)K;
    for (int shift = 24; shift >= 0; shift -= 8) {
        sc.hist[tid] = 0u;
        __syncthreads();
        for (int p = tid; p < n; p += kTopBlock) {
            const uint32_t k = key[p];
            if ((k & mask) == prefix) atomicAdd(&sc.hist[(k >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t acc = 0, d = 0;
            for (; d < 255u; ++d) {
                if (acc + sc.hist[d] >= need) break;
                acc += sc.hist[d];
            }
            sc.need = need - acc;
            sc.prefix = prefix | (d << shift);
        }
        __syncthreads();
        need = sc.need;
        prefix = sc.prefix;
        mask |= 255u << shift;
        __syncthreads();
    }
    // order-preserving compaction: thread t owns the indices [t chunk, (t + 1) chunk)
    const int chunk = (n + kTopBlock - 1) / kTopBlock;
    const int b0 = min(tid * chunk, n), b1 = min(b0 + chunk, n);
    uint32_t n_less = 0, n_eq = 0;
    for (int p = b0; p < b1; ++p) {
        n_less += key[p] < prefix;
        n_eq += key[p] == prefix;
    }
    uint32_t less = block_exclusive_scan(n_less, sc.scan[0]);
    uint32_t eq = block_exclusive_scan(n_eq, sc.scan[1]);
    for (int p = b0; p < b1; ++p) {
        const uint32_t k = key[p];
        if (k < prefix || (k == prefix && eq < need)) out[less + min(eq, need)] = (uint32_t)p;
        less += k < prefix;
        eq += k == prefix;
    }
}

// Search budget: the rigid score of every start of one ligand (the same arithmetic as the screen's
// rigid placement), then the K lowest, ties to the lower start, by a radix select over the ordered
// 32-bit scores (a start's index is its position).  Writes the chosen starts in increasing order to
// sel[lig][K]; with start_scores given, first sets every start's entry to +inf (the screen then
// writes the searched ones).
template <int BOUNDARY, int LAYOUT>
__global__ __launch_bounds__(kTopBlock) void k_rigid_top(ScreenArgs A, uint32_t *sel) {
    extern __shared__ __align__(16) char smem[];
    LigLDS &L = *reinterpret_cast<LigLDS *>(smem);
    uint32_t *key = reinterpret_cast<uint32_t *>(smem + ((sizeof(LigLDS) + 15) & ~size_t(15)));  // [QT]
    __shared__ SelectScratch sc;
    __shared__ float clash_s;
    const int lig = blockIdx.x, tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    const int QT = A.s.QT, K = A.s.top;
    load_ligand(L, A.pk, lig, A.g, tid, kTopBlock);
    if (A.start_scores)
        for (int p = tid; p < QT; p += kTopBlock) A.start_scores[(size_t)lig * QT + p] = INFINITY;
    __syncthreads();
    if (L.status != DOCK_LIG_OK) return;  // block-uniform
    if (w == 0) {
        const float c = rigid_clash(L, A.s);
        if (lane == 0) clash_s = c;
    }
    __syncthreads();
    const float clash_ref = clash_s;
    const rsrc_t rs = grid_rsrc(A.g);
    for (int p = w; p < QT; p += kTopBlock / kWave) {
        float cx[2], cy[2], cz[2];
        place(A.g, A.s, L, p, cx, cy, cz);
        float eg = 0.0f;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = lane + kWave * h;
            if (i < L.n) eg += lookup_lane<BOUNDARY, LAYOUT>(A.g, rs, L.tof[i], cx[h], cy[h], cz[h]);
        }
        const float E = wave_sum(eg) + clash_ref;
        if (lane == 0) key[p] = float_to_ordered(E);
    }
    __syncthreads();
    block_select_lowest(key, QT, K, sel + (size_t)lig * K, sc);
}

template <int APL, int BOUNDARY, int LAYOUT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_screen(ScreenArgs A) {
    extern __shared__ __align__(16) char smem[];
    LigLDS &L = *reinterpret_cast<LigLDS *>(smem);
    WaveLDS *Wv = reinterpret_cast<WaveLDS *>(smem + ((sizeof(LigLDS) + 15) & ~size_t(15)));
    __shared__ int64_t item_s;
    __shared__ uint64_t wbest_s[8];
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    WaveLDS &W = Wv[w];
    float cs[APL], sn[APL];
    angle_table<APL>(A.s.S, cs, sn);
    const rsrc_t rs = grid_rsrc(A.g);

    for (;;) {
        if (tid == 0) item_s = (int64_t)atomicAdd(A.counter, 1ull);
        __syncthreads();
        const int64_t item = item_s;
        if (item >= A.n_items) break;
        // items run batch-major: batch b of every ligand (in cost order) before batch b + 1
        const int batch = (int)(item / A.n_lig), slot = (int)(item - (int64_t)batch * A.n_lig);
        const int lig = (int)(uint32_t)A.order[slot];
        load_ligand(L, A.pk, lig, A.g, tid, blockDim.x);
        __syncthreads();
        if (L.status == DOCK_LIG_OK) {
            const float clash_ref = rigid_clash(L, A.s);
            uint64_t wbest = ~0ull;
            const int p0 = batch * A.P, p1 = min(p0 + A.P, A.s.top ? A.s.top : A.s.N);
            for (int idx = p0 + w; idx < p1; idx += A.nw) {
                // the searched starts are enumerated restart by restart, each rigid start set
                // translation-major (idx = r QT + it n_quat + iq)
                const int rq = A.s.restarts ? idx % A.s.QT : idx;
                const int p = A.s.top ? (int)A.sel[(size_t)lig * A.s.top + idx]
                                      : idx - rq + (rq % A.s.n_quat) * A.s.n_trans + rq / A.s.n_quat;
                int step = 0;
                const float E = run_start<APL, BOUNDARY, LAYOUT>(A.g, rs, A.s, L, W, p, clash_ref, cs, sn, step);
                const uint64_t key = ((uint64_t)float_to_ordered(E) << 32) | (uint32_t)p;
                wbest = key < wbest ? key : wbest;
                if (A.start_scores && lane == 0) A.start_scores[(size_t)lig * A.s.N + p] = E;
                if (A.start_steps && lane < DOCK_MAX_TORSIONS)
                    A.start_steps[((size_t)lig * A.s.N + p) * DOCK_MAX_TORSIONS + lane] =
                        (uint16_t)(lane < L.B ? step : 0);
            }
            if (lane == 0) wbest_s[w] = wbest;
        }
        __syncthreads();
        if (tid == 0 && L.status == DOCK_LIG_OK) {
            uint64_t b = wbest_s[0];
            for (int q = 1; q < A.nw; ++q) b = wbest_s[q] < b ? wbest_s[q] : b;
            atomicMin((unsigned long long *)&A.best_key[lig], (unsigned long long)b);
        }
        __syncthreads();
    }
}

// Reruns each ligand's winning start to recover its torsion steps, then writes the outputs.
template <int APL, int BOUNDARY, int LAYOUT>
__global__ __launch_bounds__(64) void k_replay(ScreenArgs A, float *best_score, int32_t *best_start,
                                               uint16_t *best_steps) {
    extern __shared__ __align__(16) char smem[];
    LigLDS &L = *reinterpret_cast<LigLDS *>(smem);
    WaveLDS &W = *reinterpret_cast<WaveLDS *>(smem + ((sizeof(LigLDS) + 15) & ~size_t(15)));
    const int lig = blockIdx.x, lane = lane_id();
    float cs[APL], sn[APL];
    angle_table<APL>(A.s.S, cs, sn);
    const rsrc_t rs = grid_rsrc(A.g);
    load_ligand(L, A.pk, lig, A.g, lane, kWave);
    __syncthreads();
    const uint64_t key = A.best_key[lig];
    int step = 0;
    float E = INFINITY;
    int p = -1;
    if (L.status == DOCK_LIG_OK && key != ~0ull) {
        p = (int)(uint32_t)key;
        const float clash_ref = rigid_clash(L, A.s);
        E = run_start<APL, BOUNDARY, LAYOUT>(A.g, rs, A.s, L, W, p, clash_ref, cs, sn, step);
    }
    if (lane < DOCK_MAX_TORSIONS) best_steps[(size_t)lig * DOCK_MAX_TORSIONS + lane] =
        (uint16_t)(p >= 0 && lane < L.B ? step : 0);
    if (lane == 0) {
        best_score[lig] = E;
        best_start[lig] = p;
    }
}

// Scores explicit poses from scratch: place, apply the given steps, full grid + clash sum.
template <int BOUNDARY, int LAYOUT>
__global__ __launch_bounds__(64) void k_score_poses(GridC g, SearchC s, PackView pk, int n_lig, const int32_t *d_lig,
                                                    const int32_t *d_start, const uint16_t *d_steps, int64_t n_poses,
                                                    float *out) {
    __shared__ LigLDS L;
    const int64_t pose = blockIdx.x;
    const int lane = lane_id();
    const int lig = d_lig[pose];
    const int p = d_start[pose];
    if (lig < 0 || lig >= n_lig || p < 0 || p >= s.N) {  // descriptor outside the library or start set
        if (lane == 0) out[pose] = NAN;
        return;
    }
    load_ligand(L, pk, lig, g, lane, kWave);
    __syncthreads();
    if (L.status != DOCK_LIG_OK) {
        if (lane == 0) out[pose] = INFINITY;
        return;
    }
    const rsrc_t rs = grid_rsrc(g);
    float cx[2], cy[2], cz[2];
    build_pose(g, s, L, p, d_steps + pose * DOCK_MAX_TORSIONS, cx, cy, cz);
    // every atom's grid term and every clash pair, from the final coordinates
    const float acc = direct_score<BOUNDARY, LAYOUT>(g, rs, s, L, cx, cy, cz);
    if (lane == 0) out[pose] = acc;
}

// ---------------------------------------------------------------------------------------------
// Pose filtering and rescoring
// ---------------------------------------------------------------------------------------------

constexpr int kMaxKeep = 16;

// The n_keep searched starts with the lowest final scores (ties to the lower start; +inf entries,
// i.e. starts not searched, are never taken), in that order; -1 where there are fewer, and for a
// ligand whose status is not OK (the screen leaves its entries unwritten).
__global__ __launch_bounds__(kTopBlock) void k_pick_poses(const LigDesc *desc, const float *start_scores, int QT,
                                                          int n_keep, int32_t *pose_start) {
    __shared__ uint32_t key[DOCK_MAX_TOP_STARTS];
    __shared__ uint32_t sel[kMaxKeep];
    __shared__ SelectScratch sc;
    const int lig = blockIdx.x, tid = threadIdx.x;
    if (desc[lig].status != DOCK_LIG_OK) {  // block-uniform
        for (int i = tid; i < n_keep; i += kTopBlock) pose_start[(size_t)lig * n_keep + i] = -1;
        return;
    }
    for (int p = tid; p < QT; p += kTopBlock) key[p] = float_to_ordered(start_scores[(size_t)lig * QT + p]);
    __syncthreads();
    const int K = min(n_keep, QT);
    block_select_lowest(key, QT, K, sel, sc);
    __syncthreads();
    if (tid == 0) {
        // order by (score, start): insertion sort of at most 16
        for (int i = 1; i < K; ++i) {
            const uint32_t v = sel[i];
            int j = i - 1;
            while (j >= 0 && key[sel[j]] > key[v]) {
                sel[j + 1] = sel[j];
                --j;
            }
            sel[j + 1] = v;
        }
        const uint32_t inf_key = float_to_ordered(INFINITY);
        for (int i = 0; i < n_keep; ++i)
            pose_start[(size_t)lig * n_keep + i] = i < K && key[sel[i]] < inf_key ? (int32_t)sel[i] : -1;
    }
}

struct PoseArgs {
    ScreenArgs A;  // grid, search, pack
    const int32_t *pose_start;
    uint16_t *pose_steps;
    float *pose_score;
    int n_keep;
};

// One wavefront per (ligand, kept slot): reruns the start with the screen's code to recover its
// total turns; the final equals the screen's per-start score bit for bit.
template <int APL, int BOUNDARY, int LAYOUT>
__global__ __launch_bounds__(64) void k_pose_replay(PoseArgs R) {
    extern __shared__ __align__(16) char smem[];
    LigLDS &L = *reinterpret_cast<LigLDS *>(smem);
    WaveLDS &W = *reinterpret_cast<WaveLDS *>(smem + ((sizeof(LigLDS) + 15) & ~size_t(15)));
    const int lig = blockIdx.x / R.n_keep, slot = blockIdx.x - lig * R.n_keep, lane = lane_id();
    const ScreenArgs &A = R.A;
    const int p = R.pose_start[(size_t)lig * R.n_keep + slot];
    uint16_t *steps = R.pose_steps + ((size_t)lig * R.n_keep + slot) * DOCK_MAX_TORSIONS;
    if (p < 0) {
        if (lane < DOCK_MAX_TORSIONS) steps[lane] = 0;
        if (lane == 0) R.pose_score[(size_t)lig * R.n_keep + slot] = NAN;
        return;
    }
    float cs[APL], sn[APL];
    angle_table<APL>(A.s.S, cs, sn);
    const rsrc_t rs = grid_rsrc(A.g);
    load_ligand(L, A.pk, lig, A.g, lane, kWave);
    __syncthreads();
    int step = 0;
    const float E = run_start<APL, BOUNDARY, LAYOUT>(A.g, rs, A.s, L, W, p, rigid_clash(L, A.s), cs, sn, step);
    if (lane < DOCK_MAX_TORSIONS) steps[lane] = (uint16_t)(lane < L.B ? step : 0);
    if (lane == 0) R.pose_score[(size_t)lig * R.n_keep + slot] = E;
}

struct RescoreArgs {
    GridC g;
    SearchC s;
    PackView pk;
    const float *prot_xyz;
    const int32_t *prot_type;
    int n_prot;
    // per type: radius, square root of the well depth, charge; the pair terms are R_a + R_b,
    // sqrt(eps_a) sqrt(eps_b) and coulomb_k q_a q_b
    double R[DOCK_MAX_TYPES], se[DOCK_MAX_TYPES], q[DOCK_MAX_TYPES];
    double coulomb_k, cap, r_min, h, ox, oy, oz, rmsd2_min, clash_cut, clash_w;
    int n_keep;
    const int32_t *pose_start;
    const uint16_t *pose_steps;
    float *pose_rescore, *best_rescore;
    int32_t *best_pose;
    double *pose_xyz;  // optional [n_lig][n_keep][128][3]
};

constexpr int kProtTile = 256;

// One wavefront per ligand: rebuilds its kept-slot poses in docking order (the k_score_poses code),
// drops a pose within rmsd_min of an earlier kept one, and rescores the rest in FP64 at the atoms'
// own positions (protein atoms staged in LDS), then picks the best.
__global__ __launch_bounds__(64) void k_filter_rescore(RescoreArgs R) {
    __shared__ LigLDS L;
    __shared__ float4 kept_xyz[kMaxKeep][DOCK_MAX_ATOMS];  // grid units
    __shared__ float4 prot[kProtTile];
    __shared__ double prot_R[kProtTile], prot_se[kProtTile], prot_q[kProtTile];
    const int lig = blockIdx.x, lane = lane_id();
    load_ligand(L, R.pk, lig, R.g, lane, kWave);
    __syncthreads();
    float best = INFINITY;
    int best_i = -1, n_kept = 0;
    for (int i = 0; i < R.n_keep; ++i) {
        const size_t slot = (size_t)lig * R.n_keep + i;
        const int p = R.pose_start[slot];
        if (p < 0 || L.status != DOCK_LIG_OK) {
            if (lane == 0) R.pose_rescore[slot] = NAN;
            continue;
        }
        // the pose, as k_score_poses builds it (grid units)
        const int n = L.n;
        float cx[2], cy[2], cz[2];
        build_pose(R.g, R.s, L, p, R.pose_steps + slot * DOCK_MAX_TORSIONS, cx, cy, cz);
        // world coordinates in FP64: x = origin + h u
        double wx[2], wy[2], wz[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            wx[h] = fma((double)cx[h], R.h, R.ox);
            wy[h] = fma((double)cy[h], R.h, R.oy);
            wz[h] = fma((double)cz[h], R.h, R.oz);
        }
        // the RMSD to every earlier kept pose (squared, Angstrom^2, FP64 sums)
        bool keep = true;
        for (int j = 0; j < n_kept; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int a = lane + kWave * h;
                if (a < n) {
                    const float4 y = kept_xyz[j][a];
                    const double dx = (double)(cx[h] - y.x), dy = (double)(cy[h] - y.y), dz = (double)(cz[h] - y.z);
                    acc += dx * dx + dy * dy + dz * dz;
                }
            }
            const double msd = wave_sum_d(acc) * R.h * R.h / n;
            if (msd < R.rmsd2_min) keep = false;
        }
        if (!keep) {
            if (lane == 0) R.pose_rescore[slot] = NAN;
            continue;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int a = lane + kWave * h;
            if (a < n) kept_xyz[n_kept][a] = make_float4(cx[h], cy[h], cz[h], 0.0f);
        }
        ++n_kept;
        if (R.pose_xyz) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int a = lane + kWave * h;
                if (a < n) {
                    double *o = R.pose_xyz + (slot * DOCK_MAX_ATOMS + a) * 3;
                    o[0] = wx[h];
                    o[1] = wy[h];
                    o[2] = wz[h];
                }
            }
        }
        // per atom: capped FP64 sum over the protein atoms
        double sum[2] = {0.0, 0.0};
        for (int base = 0; base < R.n_prot; base += kProtTile) {
            __syncthreads();
            for (int q = lane; q < kProtTile && base + q < R.n_prot; q += kWave) {
                const int j = base + q, tb = min(max(R.prot_type[j], 0), DOCK_MAX_TYPES - 1);
                prot[q] = make_float4(R.prot_xyz[3 * j], R.prot_xyz[3 * j + 1], R.prot_xyz[3 * j + 2], 0.0f);
                prot_R[q] = R.R[tb];
                prot_se[q] = R.se[tb];
                prot_q[q] = R.q[tb];
            }
            __syncthreads();
            const int cnt = min(kProtTile, R.n_prot - base);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int a = lane + kWave * h;
                if (a >= n) continue;
                const int ta = L.tof[a] / R.g.type_bytes;
                const double Ra = R.R[ta], sea = R.se[ta], kqa = R.coulomb_k * R.q[ta];
                for (int q = 0; q < cnt; ++q) {
                    const float4 pa = prot[q];
                    const double dx = wx[h] - (double)pa.x, dy = wy[h] - (double)pa.y, dz = wz[h] - (double)pa.z;
                    const double r = sqrt(dx * dx + dy * dy + dz * dz);
                    const double rt = r > R.r_min ? r : R.r_min;
                    const double sr = (Ra + prot_R[q]) / rt, s2 = sr * sr, s6 = s2 * s2 * s2;
                    sum[h] += sea * prot_se[q] * (s6 * s6 - 2.0 * s6) + kqa * prot_q[q] / (rt * rt);
                }
            }
        }
        double e = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (lane + kWave * h < n) e += sum[h] < R.cap ? sum[h] : R.cap;
        // the intra-ligand clash term, FP64 from the same coordinates
        for (int a = 0; a < n; ++a) {
            const double xa = __shfl(a < kWave ? wx[0] : wx[1], a & 63), ya = __shfl(a < kWave ? wy[0] : wy[1], a & 63),
                         za = __shfl(a < kWave ? wz[0] : wz[1], a & 63);
            const uint4 ex = L.excl[a];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int b = lane + kWave * h;
                if (b > a && b < n && !mask_has(ex, b)) {
                    const double dx = wx[h] - xa, dy = wy[h] - ya, dz = wz[h] - za;
                    const double d = sqrt(dx * dx + dy * dy + dz * dz);
                    if (d < R.clash_cut) e += R.clash_w * (R.clash_cut - d) * (R.clash_cut - d);
                }
            }
        }
        const double tot = wave_sum_d(e);
        if (lane == 0) R.pose_rescore[slot] = (float)tot;
        if ((float)tot < best) {
            best = (float)tot;
            best_i = i;
        }
    }
    if (lane == 0) {
        R.best_rescore[lig] = best;
        R.best_pose[lig] = best_i;
    }
}

// ---------------------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------------------

static GridC make_grid(const dock_grid_desc *d, const float *G) {
    GridC g;
    g.G = G;
    g.nx = d->nx;
    g.ny = d->ny;
    g.nz = d->nz;
    g.type_bytes = (uint32_t)grid_type_bytes(d);
    g.total_bytes = g.type_bytes * (uint32_t)d->n_types;
    g.row = 4u * (uint32_t)d->nx;
    g.plane = 4u * (uint32_t)(d->nx * d->ny);
    g.frow = (float)g.row;
    g.fplane = (float)g.plane;
    g.geo = Xy4Geom::of(d->nx, d->ny, d->nz);
    g.ky = 64u * g.geo.nxp - 32u;
    g.kz = 64u * g.geo.nxp * g.geo.nby - 64u;
    g.inv_h = 1.0f / d->spacing;
    g.ox_h = d->origin[0] / d->spacing;
    g.oy_h = d->origin[1] / d->spacing;
    g.oz_h = d->origin[2] / d->spacing;
    g.mx = (float)(d->nx - 1);
    g.my = (float)(d->ny - 1);
    g.mz = (float)(d->nz - 1);
    g.in_lo = kEdge;
    g.in_x = g.mx - kEdge;
    g.in_y = g.my - kEdge;
    g.in_z = g.mz - kEdge;
    g.cx = (float)(d->nx - 2);
    g.cy = (float)(d->ny - 2);
    g.cz = (float)(d->nz - 2);
    g.w_h2 = d->w_out * d->spacing * d->spacing;
    return g;
}

static int check_search(const dock_search *s) {
    LIGATE_REQUIRE(s != nullptr, DOCK_ERR_INVALID_ARG, "search is NULL");
    LIGATE_REQUIRE(s->n_quat >= 1 && s->n_trans >= 1 && s->d_quat && s->d_trans, DOCK_ERR_INVALID_ARG,
                   "empty or NULL start sets");
    LIGATE_REQUIRE((int64_t)s->n_quat * s->n_trans < (1ll << 31), DOCK_ERR_LIMIT, "too many starts");
    LIGATE_REQUIRE(s->n_steps >= 1 && s->n_steps <= DOCK_MAX_STEPS, DOCK_ERR_LIMIT, "n_steps must be in [1, 1024]");
    LIGATE_REQUIRE(s->clash_cut >= 0.0f && s->clash_w >= 0.0f, DOCK_ERR_INVALID_ARG, "negative clash parameters");
    LIGATE_REQUIRE(s->starts_per_item >= 0 && s->waves_per_block >= 0 && s->waves_per_block <= 8,
                   DOCK_ERR_INVALID_ARG, "bad tuning fields");
    LIGATE_REQUIRE(s->sweep_top >= 0 && s->passes >= 0 && s->passes <= DOCK_MAX_PASSES, DOCK_ERR_INVALID_ARG,
                   "sweep_top must be >= 0 and passes in [0, %d]", DOCK_MAX_PASSES);
    LIGATE_REQUIRE(s->sweep_top == 0 || s->sweep_top >= (int64_t)s->n_quat * s->n_trans ||
                       (int64_t)s->n_quat * s->n_trans <= DOCK_MAX_TOP_STARTS,
                   DOCK_ERR_LIMIT, "selecting sweep_top starts needs n_quat * n_trans <= %d", DOCK_MAX_TOP_STARTS);
    LIGATE_REQUIRE(s->restarts >= 0 && s->restarts <= DOCK_MAX_RESTARTS, DOCK_ERR_INVALID_ARG,
                   "restarts must be in [0, %d]", DOCK_MAX_RESTARTS);
    LIGATE_REQUIRE(s->restarts == 0 || s->d_init_steps, DOCK_ERR_INVALID_ARG, "restarts need d_init_steps");
    LIGATE_REQUIRE(s->restarts == 0 || s->sweep_top == 0, DOCK_ERR_INVALID_ARG,
                   "torsion restarts are not combined with sweep_top");
    LIGATE_REQUIRE((int64_t)s->n_quat * s->n_trans * (1 + s->restarts) < (1ll << 31), DOCK_ERR_LIMIT,
                   "too many searched starts");
    return DOCK_OK;
}

static SearchC make_search(const dock_search *d, float spacing) {
    SearchC s;
    s.quat = d->d_quat;
    s.trans = d->d_trans;
    s.n_quat = d->n_quat;
    s.n_trans = d->n_trans;
    s.S = d->n_steps;
    s.QT = d->n_quat * d->n_trans;
    s.cut = d->clash_cut / spacing;
    // a lane whose d2 is below (cut + margin)^2 is evaluated; beyond it the penalty is zero
    s.cut2 = (s.cut + 1e-3f) * (s.cut + 1e-3f);
    const float keep = s.cut + 1e-3f;  // pairs this close somewhere on the circle are kept
    s.cut2_keep = keep * keep;
    s.w = d->clash_w * spacing * spacing;
    s.sw = sqrtf(s.w);
    s.swc = s.sw * s.cut;
    s.top = d->sweep_top > 0 && d->sweep_top < s.QT ? d->sweep_top : 0;
    s.passes = d->passes > 1 ? d->passes : 1;
    s.restarts = d->restarts;
    s.N = s.QT * (1 + d->restarts);
    s.init = d->d_init_steps;
    return s;
}

static size_t al(size_t v) { return (v + 255) & ~size_t(255); }

static size_t screen_lds(int nw) { return ((sizeof(LigLDS) + 15) & ~size_t(15)) + sizeof(WaveLDS) * (size_t)nw; }

// Compute units of the calling thread's current device (queried per call: the device may change
// between calls, and the query costs far less than a launch).
static int default_cu_count() {
    int dev = 0, cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    return cu > 0 ? cu : 256;
}

template <int APL, int BOUNDARY, int LAYOUT>
static int launch_screen(const ScreenArgs &A, float *bs, int32_t *bp, uint16_t *bst, hipStream_t st) {
    if (A.s.top) {
        const size_t lds = ((sizeof(LigLDS) + 15) & ~size_t(15)) + 4 * (size_t)A.s.QT;
        hipLaunchKernelGGL((k_rigid_top<BOUNDARY, LAYOUT>), dim3((unsigned)A.n_lig), dim3(kTopBlock), lds, st, A,
                           const_cast<uint32_t *>(A.sel));
    }
    const int cu = default_cu_count();
    const size_t lds = screen_lds(A.nw);
    int per_cu = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&k_screen<APL, BOUNDARY, LAYOUT>),
                                                 kWave * A.nw, lds);
    if (per_cu <= 0) per_cu = 1;
    const int64_t blocks = std::min<int64_t>(A.n_items, (int64_t)cu * per_cu);
    if (blocks > 0)
        hipLaunchKernelGGL((k_screen<APL, BOUNDARY, LAYOUT>), dim3((unsigned)blocks), dim3(kWave * A.nw), lds, st, A);
    hipLaunchKernelGGL((k_replay<APL, BOUNDARY, LAYOUT>), dim3((unsigned)A.n_lig), dim3(kWave), screen_lds(1), st, A, bs, bp,
                       bst);
    return check_launch("dock_screen");
}

template <int BOUNDARY, int LAYOUT>
static int dispatch_apl(int S, const ScreenArgs &A, float *bs, int32_t *bp, uint16_t *bst, hipStream_t st) {
    if (S <= 64) return launch_screen<1, BOUNDARY, LAYOUT>(A, bs, bp, bst, st);
    if (S <= 128) return launch_screen<2, BOUNDARY, LAYOUT>(A, bs, bp, bst, st);
    if (S <= 256) return launch_screen<4, BOUNDARY, LAYOUT>(A, bs, bp, bst, st);
    if (S <= 512) return launch_screen<8, BOUNDARY, LAYOUT>(A, bs, bp, bst, st);
    return launch_screen<16, BOUNDARY, LAYOUT>(A, bs, bp, bst, st);
}

template <int LAYOUT>
static int dispatch_boundary(int boundary, int S, const ScreenArgs &A, float *bs, int32_t *bp, uint16_t *bst,
                             hipStream_t st) {
    if (boundary == DOCK_BOUNDARY_PERIODIC) return dispatch_apl<DOCK_BOUNDARY_PERIODIC, LAYOUT>(S, A, bs, bp, bst, st);
    return dispatch_apl<DOCK_BOUNDARY_CLAMP, LAYOUT>(S, A, bs, bp, bst, st);
}

template <int APL, int BOUNDARY, int LAYOUT>
static void launch_pose_replay(const PoseArgs &R, int n_lig, hipStream_t st) {
    hipLaunchKernelGGL((k_pose_replay<APL, BOUNDARY, LAYOUT>), dim3((unsigned)(n_lig * R.n_keep)), dim3(kWave),
                       screen_lds(1), st, R);
}

template <int BOUNDARY, int LAYOUT>
static void replay_apl(int S, const PoseArgs &R, int n_lig, hipStream_t st) {
    if (S <= 64) return launch_pose_replay<1, BOUNDARY, LAYOUT>(R, n_lig, st);
    if (S <= 128) return launch_pose_replay<2, BOUNDARY, LAYOUT>(R, n_lig, st);
    if (S <= 256) return launch_pose_replay<4, BOUNDARY, LAYOUT>(R, n_lig, st);
    if (S <= 512) return launch_pose_replay<8, BOUNDARY, LAYOUT>(R, n_lig, st);
    return launch_pose_replay<16, BOUNDARY, LAYOUT>(R, n_lig, st);
}

}  // namespace ligate

using namespace ligate;

namespace ligate {

// Checks the screen's arguments that decide its workspace and returns the workspace size.
static int screen_ws_need(const dock_grid_desc *gd, const dock_search *sd, int32_t n_lig, int64_t n_atoms_total,
                          size_t *need) {
    int rc = grid_desc_check(gd);
    if (rc) return rc;
    rc = check_search(sd);
    if (rc) return rc;
    LIGATE_REQUIRE(n_lig >= 1 && n_atoms_total >= 0 && n_atoms_total < (1ll << 31), DOCK_ERR_INVALID_ARG,
                   "bad library size");
    const SearchC sc = make_search(sd, gd->spacing);
    const size_t sel_bytes = sc.top ? al(4 * (size_t)n_lig * (size_t)sc.top) : 0;
    *need = al(8 * (size_t)n_lig) + al(8 * (size_t)n_lig) + al(256) + sel_bytes + radix_sort_ws_bytes(n_lig);
    return DOCK_OK;
}

// Enqueues a screen whose arguments screen_ws_need accepted, with a workspace of at least that size.
static int screen_enqueue(const dock_grid_desc *gd, const float *d_grids, const void *d_pack, int32_t n_lig,
                          int64_t n_atoms_total, const dock_search *sd, float *d_best_score, int32_t *d_best_start,
                          uint16_t *d_best_steps, float *d_start_scores, uint16_t *d_start_steps,
                          uint64_t *d_pose_count, void *d_ws, hipStream_t st) {
    LIGATE_REQUIRE(d_grids && d_pack && d_best_score && d_best_start && d_best_steps, DOCK_ERR_INVALID_ARG,
                   "NULL array");
    const SearchC sc = make_search(sd, gd->spacing);
    const size_t sel_bytes = sc.top ? al(4 * (size_t)n_lig * (size_t)sc.top) : 0;
    char *w = (char *)d_ws;
    uint64_t *best_key = (uint64_t *)w;
    uint64_t *order = (uint64_t *)(w + al(8 * (size_t)n_lig));
    unsigned long long *counter = (unsigned long long *)(w + 2 * al(8 * (size_t)n_lig));
    uint32_t *sel = sc.top ? (uint32_t *)(w + 2 * al(8 * (size_t)n_lig) + al(256)) : nullptr;
    void *rws = w + 2 * al(8 * (size_t)n_lig) + al(256) + sel_bytes;

    ScreenArgs A;
    A.g = make_grid(gd, d_grids);
    A.g.G = d_grids;
    A.s = sc;
    A.pk = PackView::of(d_pack, n_lig, n_atoms_total);
    A.sel = sel;
    A.order = order;
    A.best_key = best_key;
    A.counter = counter;
    A.start_scores = d_start_scores;
    A.start_steps = d_start_steps;
    A.n_lig = n_lig;
    A.nw = sd->waves_per_block ? sd->waves_per_block : 4;
    LIGATE_REQUIRE(A.nw == 1 || A.nw == 2 || A.nw == 4 || A.nw == 8, DOCK_ERR_INVALID_ARG,
                   "waves_per_block must be 1, 2, 4 or 8");
    int P = sd->starts_per_item;
    if (P == 0) {
        // enough items to keep every block busy several times over, at most 256 starts per item
        const int64_t slots = (int64_t)default_cu_count() * 6;
        const int64_t total = (int64_t)n_lig * (A.s.top ? A.s.top : A.s.N);
        int64_t want = total / (4 * slots);
        want = std::max<int64_t>(A.nw, std::min<int64_t>(256, want));
        P = (int)want;
    }
    const int n_searched = A.s.top ? A.s.top : A.s.N;
    P = std::min(P, n_searched);
    A.P = P;
    A.bpl = (n_searched + P - 1) / P;
    A.n_items = (int64_t)n_lig * A.bpl;

    // the workspace is cleared by a kernel (best keys, the work counter, the pose count), never by
    // a memset, so a captured or repeated call starts from zero
    const unsigned nb = (unsigned)((n_lig + 255) / 256);
    hipLaunchKernelGGL(k_screen_init, dim3(nb), dim3(256), 0, st, best_key, n_lig, counter, d_pose_count);
    // every rigid start is scored once when starts are selected, every searched start's first pose otherwise
    hipLaunchKernelGGL(k_screen_plan, dim3(nb), dim3(256), 0, st, A.pk.desc, n_lig, A.s.S, order, d_pose_count,
                       A.s.top ? A.s.QT : A.s.N, n_searched, A.s.passes);
    int rc = radix_sort_u64(order, n_lig, 32, 64, rws, st);
    if (rc) return rc;
    if (gd->layout == DOCK_LAYOUT_XY4)
        return dispatch_boundary<DOCK_LAYOUT_XY4>(gd->boundary, A.s.S, A, d_best_score, d_best_start, d_best_steps, st);
    return dispatch_boundary<DOCK_LAYOUT_LINEAR>(gd->boundary, A.s.S, A, d_best_score, d_best_start, d_best_steps, st);
}

// Scratch of dock_screen_noalloc: one copy per GPU, allocated with the code object and held
// until the process ends.  Host code never uses this name as an address: the device address of
// each GPU's copy comes from hipGetSymbolAddress (noalloc_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[DOCK_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch, looked up once per device with that device current.
static int noalloc_scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_last_error("dock_screen_noalloc: hipGetDevice: %s", hipGetErrorString(e));
        return DOCK_ERR_HIP;
    }
    LIGATE_REQUIRE(dev >= 0 && dev < kMaxDevices, DOCK_ERR_LIMIT, "device %d beyond %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            set_last_error("dock_screen_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return DOCK_ERR_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DOCK_OK;
}

}  // namespace ligate

extern "C" int dock_screen(const dock_grid_desc *gd, const float *d_grids, const void *d_pack, int32_t n_lig,
                           int64_t n_atoms_total, const dock_search *sd, float *d_best_score, int32_t *d_best_start,
                           uint16_t *d_best_steps, float *d_start_scores, uint16_t *d_start_steps,
                           uint64_t *d_pose_count, void *d_ws,
                           size_t *ws_bytes, void *stream) {
    LIGATE_ABI_RANGE();
    size_t need = 0;
    int rc = screen_ws_need(gd, sd, n_lig, n_atoms_total, &need);
    if (rc) return rc;
    LIGATE_REQUIRE(ws_bytes != nullptr, DOCK_ERR_INVALID_ARG, "ws_bytes is NULL");
    if (d_ws == nullptr) {
        *ws_bytes = need;
        return DOCK_OK;
    }
    LIGATE_REQUIRE(*ws_bytes >= need, DOCK_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", *ws_bytes, need);
    return screen_enqueue(gd, d_grids, d_pack, n_lig, n_atoms_total, sd, d_best_score, d_best_start, d_best_steps,
                          d_start_scores, d_start_steps, d_pose_count, d_ws, (hipStream_t)stream);
}

extern "C" int dock_screen_noalloc(const dock_grid_desc *gd, const float *d_grids, const void *d_pack, int32_t n_lig,
                                   int64_t n_atoms_total, const dock_search *sd, float *d_best_score,
                                   int32_t *d_best_start, uint16_t *d_best_steps, float *d_start_scores,
                                   uint16_t *d_start_steps, uint64_t *d_pose_count, void *stream) {
    LIGATE_ABI_RANGE();
    size_t need = 0;
    int rc = screen_ws_need(gd, sd, n_lig, n_atoms_total, &need);
    if (rc) return rc;
    LIGATE_REQUIRE(need <= (size_t)DOCK_NOALLOC_SCRATCH_BYTES, DOCK_ERR_LIMIT,
                   "this screen needs %zu bytes of scratch, the allocation-free entry point has %zu", need,
                   (size_t)DOCK_NOALLOC_SCRATCH_BYTES);
    LIGATE_REQUIRE(d_grids && d_pack && d_best_score && d_best_start && d_best_steps, DOCK_ERR_INVALID_ARG,
                   "NULL array");
    void *ptr = nullptr;
    rc = noalloc_scratch_ptr(&ptr);
    if (rc) return rc;
    return screen_enqueue(gd, d_grids, d_pack, n_lig, n_atoms_total, sd, d_best_score, d_best_start, d_best_steps,
                          d_start_scores, d_start_steps, d_pose_count, ptr, (hipStream_t)stream);
}

extern "C" int dock_score_poses(const dock_grid_desc *gd, const float *d_grids, const void *d_pack, int32_t n_lig,
                                int64_t n_atoms_total, const dock_search *sd, const int32_t *d_lig,
                                const int32_t *d_start, const uint16_t *d_steps, int64_t n_poses, float *d_scores,
                                void *stream) {
    LIGATE_ABI_RANGE();
    int rc = grid_desc_check(gd);
    if (rc) return rc;
    rc = check_search(sd);
    if (rc) return rc;
    LIGATE_REQUIRE(n_lig >= 1 && n_poses >= 0 && n_poses < (1ll << 31), DOCK_ERR_INVALID_ARG, "bad sizes");
    if (n_poses == 0) return DOCK_OK;
    LIGATE_REQUIRE(d_grids && d_pack && d_lig && d_start && d_steps && d_scores, DOCK_ERR_INVALID_ARG, "NULL array");
    const GridC g = make_grid(gd, d_grids);
    const SearchC s = make_search(sd, gd->spacing);
    const PackView pk = PackView::of(d_pack, n_lig, n_atoms_total);
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)n_poses), block(kWave);
    const bool per = gd->boundary == DOCK_BOUNDARY_PERIODIC, xy4 = gd->layout == DOCK_LAYOUT_XY4;
    if (per && xy4)
        hipLaunchKernelGGL((k_score_poses<DOCK_BOUNDARY_PERIODIC, DOCK_LAYOUT_XY4>), grid, block, 0, st, g, s, pk,
                           n_lig, d_lig, d_start, d_steps, n_poses, d_scores);
    else if (per)
        hipLaunchKernelGGL((k_score_poses<DOCK_BOUNDARY_PERIODIC, DOCK_LAYOUT_LINEAR>), grid, block, 0, st, g, s, pk,
                           n_lig, d_lig, d_start, d_steps, n_poses, d_scores);
    else if (xy4)
        hipLaunchKernelGGL((k_score_poses<DOCK_BOUNDARY_CLAMP, DOCK_LAYOUT_XY4>), grid, block, 0, st, g, s, pk, n_lig,
                           d_lig, d_start, d_steps, n_poses, d_scores);
    else
        hipLaunchKernelGGL((k_score_poses<DOCK_BOUNDARY_CLAMP, DOCK_LAYOUT_LINEAR>), grid, block, 0, st, g, s, pk,
                           n_lig, d_lig, d_start, d_steps, n_poses, d_scores);
    return check_launch("dock_score_poses");
}

extern "C" int dock_rescore(const dock_grid_desc *gd, const float *d_grids, const void *d_pack, int32_t n_lig,
                            int64_t n_atoms_total, const dock_search *sd, const float *d_start_scores,
                            const float *d_prot_xyz, const int32_t *d_prot_type, int32_t n_prot,
                            const dock_type_param *h_params, const dock_potential *pot, int32_t n_keep,
                            float rmsd_min, int32_t *d_pose_start, uint16_t *d_pose_steps, float *d_pose_score,
                            float *d_pose_rescore, float *d_best_rescore, int32_t *d_best_pose, double *d_pose_xyz,
                            void *stream) {
    LIGATE_ABI_RANGE();
    int rc = grid_desc_check(gd);
    if (rc) return rc;
    rc = check_search(sd);
    if (rc) return rc;
    LIGATE_REQUIRE(n_lig >= 1 && n_atoms_total >= 0 && n_atoms_total < (1ll << 31), DOCK_ERR_INVALID_ARG,
                   "bad library size");
    LIGATE_REQUIRE(n_keep >= 1 && n_keep <= kMaxKeep, DOCK_ERR_INVALID_ARG, "n_keep must be in [1, %d]", kMaxKeep);
    LIGATE_REQUIRE(rmsd_min >= 0.0f, DOCK_ERR_INVALID_ARG, "rmsd_min must be >= 0");
    LIGATE_REQUIRE((int64_t)sd->n_quat * sd->n_trans * (1 + sd->restarts) <= DOCK_MAX_TOP_STARTS, DOCK_ERR_LIMIT,
                   "picking poses needs at most %d searched starts", DOCK_MAX_TOP_STARTS);
    LIGATE_REQUIRE(n_prot >= 0 && (n_prot == 0 || (d_prot_xyz && d_prot_type)), DOCK_ERR_INVALID_ARG,
                   "protein arrays are NULL");
    LIGATE_REQUIRE(h_params && pot && pot->r_min > 0.0, DOCK_ERR_INVALID_ARG, "bad potential");
    LIGATE_REQUIRE(d_grids && d_pack && d_start_scores && d_pose_start && d_pose_steps && d_pose_score &&
                       d_pose_rescore && d_best_rescore && d_best_pose,
                   DOCK_ERR_INVALID_ARG, "NULL array");
    // every argument is checked before the first launch: an error leaves the stream untouched
    for (int t = 0; t < gd->n_types; ++t)
        LIGATE_REQUIRE(h_params[t].eps >= 0.0, DOCK_ERR_INVALID_ARG, "eps of type %d is negative", t);
    hipStream_t st = (hipStream_t)stream;
    ScreenArgs A{};
    A.g = make_grid(gd, d_grids);
    A.s = make_search(sd, gd->spacing);
    A.pk = PackView::of(d_pack, n_lig, n_atoms_total);
    A.n_lig = n_lig;
    hipLaunchKernelGGL(k_pick_poses, dim3((unsigned)n_lig), dim3(kTopBlock), 0, st, A.pk.desc, d_start_scores,
                       A.s.N, n_keep, d_pose_start);
    PoseArgs R{A, d_pose_start, d_pose_steps, d_pose_score, n_keep};
    const bool per = gd->boundary == DOCK_BOUNDARY_PERIODIC, xy4 = gd->layout == DOCK_LAYOUT_XY4;
    if (per && xy4) replay_apl<DOCK_BOUNDARY_PERIODIC, DOCK_LAYOUT_XY4>(A.s.S, R, n_lig, st);
    else if (per) replay_apl<DOCK_BOUNDARY_PERIODIC, DOCK_LAYOUT_LINEAR>(A.s.S, R, n_lig, st);
    else if (xy4) replay_apl<DOCK_BOUNDARY_CLAMP, DOCK_LAYOUT_XY4>(A.s.S, R, n_lig, st);
    else replay_apl<DOCK_BOUNDARY_CLAMP, DOCK_LAYOUT_LINEAR>(A.s.S, R, n_lig, st);
    RescoreArgs Q{};
    Q.g = A.g;
    Q.s = A.s;
    Q.pk = A.pk;
    Q.prot_xyz = d_prot_xyz;
    Q.prot_type = d_prot_type;
    Q.n_prot = n_prot;
    for (int t = 0; t < DOCK_MAX_TYPES; ++t) {
        const dock_type_param p = t < gd->n_types ? h_params[t] : dock_type_param{1.0, 0.0, 0.0};
        Q.R[t] = p.R;
        Q.se[t] = sqrt(p.eps);
        Q.q[t] = p.q;
    }
    Q.coulomb_k = pot->coulomb_k;
    Q.cap = pot->cap;
    Q.r_min = pot->r_min;
    Q.h = gd->spacing;
    Q.ox = gd->origin[0];
    Q.oy = gd->origin[1];
    Q.oz = gd->origin[2];
    Q.rmsd2_min = (double)rmsd_min * (double)rmsd_min;
    Q.clash_cut = sd->clash_cut;
    Q.clash_w = sd->clash_w;
    Q.n_keep = n_keep;
    Q.pose_start = d_pose_start;
    Q.pose_steps = d_pose_steps;
    Q.pose_rescore = d_pose_rescore;
    Q.best_rescore = d_best_rescore;
    Q.best_pose = d_best_pose;
    Q.pose_xyz = d_pose_xyz;
    hipLaunchKernelGGL(k_filter_rescore, dim3((unsigned)n_lig), dim3(kWave), 0, st, Q);
    return check_launch("dock_rescore");
}
