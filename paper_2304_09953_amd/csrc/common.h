// Internal definitions shared by the HIP sources of libligate (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>
#include <stdio.h>

#include "ligate_dock.h"

namespace ligate {

constexpr int kWave = 64;

// A roctx range named after the C ABI function it spans, opened on entry and closed on every
// return: rocprofv3 --marker-trace shows each call with the kernels it enqueued.  Without a
// profiler attached the two calls do nothing.
struct AbiRange {
    explicit AbiRange(const char *name) { roctxRangePushA(name); }
    ~AbiRange() { roctxRangePop(); }
    AbiRange(const AbiRange &) = delete;
    AbiRange &operator=(const AbiRange &) = delete;
};
#define LIGATE_ABI_RANGE() const ::ligate::AbiRange ligate_abi_range_(__func__)

// ---------------------------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------------------------

void set_last_error(const char *fmt, ...);

#define LIGATE_REQUIRE(cond, code, ...)            \
    do {                                          \
        if (!(cond)) {                            \
            ::ligate::set_last_error(__VA_ARGS__); \
            return (code);                        \
        }                                         \
    } while (0)

// Checks for a launch error after enqueueing kernels.
int check_launch(const char *what);

// ---------------------------------------------------------------------------------------------
// Grid storage
// ---------------------------------------------------------------------------------------------

// DOCK_LAYOUT_XY4 storage order: the 16-byte records are grouped in bricks of 1 x 2 x 2 records
// (64 bytes), the records of a (y, z) pair of rows; brick (x, by, bz) has index
// x + nxp (by + nby bz) with nxp = nx rounded up to even, and record (x, y, z) sits at position
// (y & 1) + 2 (z & 1) inside its brick.  A 128-byte line thus holds the 2 x 2 x 2 records of
// x = 2i, 2i + 1.  A trilinear lookup reads the records (x0, y0, z0) and (x0, y0, z0 + 1), usually
// from the same line, and the lookups of neighbouring points share lines in all three directions.
struct Xy4Geom {
    uint32_t nxp, nby, nbz;  // nx rounded up to even; ceil(ny / 2), ceil(nz / 2)

    __host__ __device__ static Xy4Geom of(int nx, int ny, int nz) {
        return Xy4Geom{(uint32_t)(nx + 1) & ~1u, (uint32_t)(ny + 1) / 2, (uint32_t)(nz + 1) / 2};
    }
    __host__ __device__ uint64_t type_bytes() const { return 64ull * nxp * nby * nbz; }
    __host__ __device__ uint32_t offset(uint32_t x, uint32_t y, uint32_t z) const {
        return 64u * (x + nxp * ((y >> 1) + nby * (z >> 1))) + 16u * ((y & 1u) + 2u * (z & 1u));
    }
};

// Bytes of one type grid in layout g->layout (the descriptor is assumed valid).
inline uint64_t grid_type_bytes(const dock_grid_desc *g) {
    if (g->layout == DOCK_LAYOUT_XY4) return Xy4Geom::of(g->nx, g->ny, g->nz).type_bytes();
    return 4ull * (uint64_t)g->nx * (uint64_t)g->ny * (uint64_t)g->nz;
}

// ---------------------------------------------------------------------------------------------
// Packed ligand library (device-resident, opaque to callers)
// ---------------------------------------------------------------------------------------------

struct LigDesc {
    int32_t atom_off;  // first atom in the SoA arrays (same as the CSR input)
    int32_t n;         // atoms
    int32_t B;         // torsions
    int32_t status;    // DOCK_LIG_*
    int32_t sum_m;     // sum over torsions of the moving-set size
    int32_t n_pairs;   // clash pairs (atoms three or more bonds apart)
    int32_t pad0, pad1;
};
static_assert(sizeof(LigDesc) == 32, "LigDesc layout");

// One torsion in sweep order: moving-atom mask, axis a -> b (a on the core side), moving count.
struct TorRec {
    uint32_t mask[4];
    uint8_t a, b;
    uint16_t m;
};
static_assert(sizeof(TorRec) == 20, "TorRec layout");

struct PackLayout {
    size_t desc, x, y, z, type, excl, tor, total;

    static inline size_t align(size_t v) { return (v + 255) & ~size_t(255); }

    static PackLayout make(int32_t n_lig, int64_t n_atoms) {
        PackLayout L;
        size_t o = 0;
        L.desc = o;  o = align(o + sizeof(LigDesc) * (size_t)n_lig);
        L.x = o;     o = align(o + sizeof(float) * (size_t)n_atoms);
        L.y = o;     o = align(o + sizeof(float) * (size_t)n_atoms);
        L.z = o;     o = align(o + sizeof(float) * (size_t)n_atoms);
        L.type = o;  o = align(o + (size_t)n_atoms);
        L.excl = o;  o = align(o + 16 * (size_t)n_atoms);
        L.tor = o;   o = align(o + sizeof(TorRec) * DOCK_MAX_TORSIONS * (size_t)n_lig);
        L.total = o;
        return L;
    }
};

// Device view of a pack.
struct PackView {
    const LigDesc *desc;
    const float *x, *y, *z;
    const uint8_t *type;
    const uint4 *excl;     // per atom: atoms fewer than three bonds away (including itself)
    const TorRec *tor;     // [n_lig][DOCK_MAX_TORSIONS]

    static PackView of(const void *base, int32_t n_lig, int64_t n_atoms) {
        PackLayout L = PackLayout::make(n_lig, n_atoms);
        const char *b = (const char *)base;
        PackView v;
        v.desc = (const LigDesc *)(b + L.desc);
        v.x = (const float *)(b + L.x);
        v.y = (const float *)(b + L.y);
        v.z = (const float *)(b + L.z);
        v.type = (const uint8_t *)(b + L.type);
        v.excl = (const uint4 *)(b + L.excl);
        v.tor = (const TorRec *)(b + L.tor);
        return v;
    }
};

// ---------------------------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------------------------

// Order-preserving map of a float to uint32 (NaN ranks as +inf, -0 as +0).
__device__ __forceinline__ uint32_t float_to_ordered(float f) {
    uint32_t b = __float_as_uint(f);
    if (f != f) b = 0x7f800000u;
    if (b == 0x80000000u) b = 0u;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float ordered_to_float(uint32_t o) {
    uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(b);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Orders LDS accesses between the lanes of one wavefront (a wave executes in lockstep,
// so this only needs to stop the compiler from moving memory operations across it).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Minimum of two values that are never NaN: one v_min_f32, without the quieting of signalling
// NaNs that fminf adds to each operand.
__device__ __forceinline__ float min_nonan(float a, float b) {
    float r;
    asm volatile("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Wave minimum of values that are never NaN.
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = min_nonan(v, __shfl_xor(v, off));
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v |= (uint32_t)__shfl_xor((int)v, off);
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Number of set bits of a 64-bit lane mask below this lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ bool mask_has(const uint4 &m, int i) {
    uint32_t w = (i < 32) ? m.x : (i < 64) ? m.y : (i < 96) ? m.z : m.w;
    return (w >> (i & 31)) & 1u;
}

// The mask with atom i's bit cleared (i wave-uniform).
__device__ __forceinline__ uint4 mask_without(uint4 m, int i) {
    const uint32_t keep = ~(1u << (i & 31));
    const int w = i >> 5;
    m.x &= w == 0 ? keep : ~0u;
    m.y &= w == 1 ? keep : ~0u;
    m.z &= w == 2 ? keep : ~0u;
    m.w &= w == 3 ? keep : ~0u;
    return m;
}

// mask_has for atom lane + 64 h of a wavefront (lane < 64; h is 0 or 1, usually a constant of an
// unrolled loop), selecting between two words instead of four.
__device__ __forceinline__ bool mask_has_lane(const uint4 &m, int h, int lane) {
    const uint32_t w = h == 0 ? (lane < 32 ? m.x : m.y) : (lane < 32 ? m.z : m.w);
    return (w >> (lane & 31)) & 1u;
}

// ---------------------------------------------------------------------------------------------
// Radix sort of 64-bit keys (stable LSD, 8-bit digits), shared by the screen planner and top-k
// ---------------------------------------------------------------------------------------------

size_t radix_sort_ws_bytes(int64_t n);
// Sorts d_keys (n entries) ascending; the result is left in d_keys.  Bits below lo_bit are
// assumed not to matter for the order requested (they are still carried).  Uses d_ws.
int radix_sort_u64(uint64_t *d_keys, int64_t n, int lo_bit, int hi_bit, void *d_ws, hipStream_t stream);

}  // namespace ligate
