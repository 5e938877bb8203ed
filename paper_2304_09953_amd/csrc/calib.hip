// Peak-calibration kernels (measurement helpers; no part of the docking method).
#include "common.h"
#include "ligate_calib.h"

namespace ligate {

constexpr int kCalibBlock = 256;

// 16 independent FMA chains per thread; the multiplier and addend keep the values bounded.
__global__ __launch_bounds__(kCalibBlock) void k_calib_fma(int iters, float a, float b, float *out) {
    const int tid = blockIdx.x * kCalibBlock + threadIdx.x;
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = (float)(tid & 255) * 1e-3f + (float)k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = fmaf(v[k], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += v[k];
    out[tid] = s;
}

// Every block streams the whole buffer `reps` times; a wavefront reads 1 KiB per step (64 lanes x
// 16 bytes), the block's four wavefronts start at different 4 KiB-aligned pieces.
__global__ __launch_bounds__(kCalibBlock) void k_calib_read(const float4 *__restrict__ buf, uint32_t n_vec, int reps,
                                                            float *out) {
    const uint32_t tid = threadIdx.x;
    const uint32_t start = (blockIdx.x * 4096u / 16u) % n_vec;  // spread blocks over the buffer
    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int r = 0; r < reps; ++r) {
        // n_vec is a multiple of 1024: every thread takes n_vec / 1024 steps of four loads
        for (uint32_t i = tid; i < n_vec; i += 4 * kCalibBlock) {
            uint32_t j0 = start + i;
            j0 -= j0 >= n_vec ? n_vec : 0u;  // start, i < n_vec
            uint32_t j1 = j0 + kCalibBlock, j2 = j0 + 2 * kCalibBlock, j3 = j0 + 3 * kCalibBlock;
            j1 -= j1 >= n_vec ? n_vec : 0u;  // j0 < n_vec and 768 < n_vec: one wrap at most
            j2 -= j2 >= n_vec ? n_vec : 0u;
            j3 -= j3 >= n_vec ? n_vec : 0u;
            const float4 x0 = buf[j0], x1 = buf[j1], x2 = buf[j2], x3 = buf[j3];
            acc.x += x0.x + x1.x + x2.x + x3.x;
            acc.y += x0.y + x1.y + x2.y + x3.y;
            acc.z += x0.z + x1.z + x2.z + x3.z;
            acc.w += x0.w + x1.w + x2.w + x3.w;
        }
    }
    out[blockIdx.x * kCalibBlock + tid] = acc.x + acc.y + acc.z + acc.w;
}

}  // namespace ligate

using namespace ligate;

extern "C" int calib_fma_f32(int32_t blocks, int32_t iters, float *d_out, void *stream) {
    LIGATE_ABI_RANGE();
    LIGATE_REQUIRE(blocks >= 1 && blocks <= (1 << 20) && iters >= 1 && iters <= (1 << 24), DOCK_ERR_INVALID_ARG,
                   "blocks or iters out of range");
    LIGATE_REQUIRE(d_out != nullptr, DOCK_ERR_INVALID_ARG, "d_out is NULL");
    hipLaunchKernelGGL(k_calib_fma, dim3((unsigned)blocks), dim3(kCalibBlock), 0, (hipStream_t)stream, iters,
                       0.999f, 1e-3f, d_out);
    return check_launch("calib_fma_f32");
}

extern "C" int calib_cache_read(const void *d_buf, size_t bytes, int32_t reps, int32_t blocks, float *d_out,
                                void *stream) {
    LIGATE_ABI_RANGE();
    LIGATE_REQUIRE(d_buf && d_out, DOCK_ERR_INVALID_ARG, "NULL argument");
    LIGATE_REQUIRE(((uintptr_t)d_buf & 15u) == 0 && bytes >= 16384 && bytes % 16384 == 0 && bytes < (1ull << 34),
                   DOCK_ERR_INVALID_ARG, "bytes must be a positive multiple of 16384 (buffer 16-byte aligned)");
    LIGATE_REQUIRE(blocks >= 1 && blocks <= (1 << 20) && reps >= 1 && reps <= (1 << 20), DOCK_ERR_INVALID_ARG,
                   "blocks or reps out of range");
    hipLaunchKernelGGL(k_calib_read, dim3((unsigned)blocks), dim3(kCalibBlock), 0, (hipStream_t)stream,
                       reinterpret_cast<const float4 *>(d_buf), (uint32_t)(bytes / 16), reps, d_out);
    return check_launch("calib_cache_read");
}
