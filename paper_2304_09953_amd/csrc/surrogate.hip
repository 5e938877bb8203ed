// Learned pre-filter: ligand features, a 3-layer MLP on the matrix cores (BF16 operands, FP32
// accumulation, v_mfma_f32_32x32x16_bf16), its backward pass and Adam.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "ligate_surrogate.h"

namespace ligate {

// ---------------------------------------------------------------------------------------------
// BF16 helpers (round to nearest even)
// ---------------------------------------------------------------------------------------------

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------------------------
// Features: one wavefront per ligand
// ---------------------------------------------------------------------------------------------

constexpr int kRows = 16, kSlots = 32, kBins = 30;

__global__ __launch_bounds__(64) void k_features(const int32_t *__restrict__ atom_off, const float *__restrict__ xyz,
                                                 const uint8_t *__restrict__ type, PackView pk,
                                                 const float *__restrict__ mean, const float *__restrict__ istd,
                                                 float *__restrict__ out_f, uint16_t *__restrict__ out_b) {
    __shared__ int cnt[kRows * kSlots];
    const int l = blockIdx.x, lane = lane_id();
    const LigDesc d = pk.desc[l];
    bool ok = d.status == DOCK_LIG_OK;
    if (ok) {
        // the histogram has one row per type below kRows: a ligand with any other type (a pack
        // built with more types) is not representable and gets zero features
        bool bad = false;
        for (int i = lane; i < d.n; i += kWave) bad |= type[atom_off[l] + i] >= kRows;
        ok = __ballot(bad) == 0ull;
    }
    for (int f = lane; f < kRows * kSlots; f += kWave) cnt[f] = 0;
    wave_sync();
    if (ok) {
        const int a0 = atom_off[l], n = d.n;
        for (int i = lane; i < n; i += kWave) {
            const int ti = type[a0 + i];
            atomicAdd(&cnt[ti * kSlots], 1);
            const float xi = xyz[3 * (a0 + i)], yi = xyz[3 * (a0 + i) + 1], zi = xyz[3 * (a0 + i) + 2];
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                // squared distance with every product and sum rounded (no contraction), so the
                // bin decision is reproducible
                const float dx = __fsub_rn(xi, xyz[3 * (a0 + j)]);
                const float dy = __fsub_rn(yi, xyz[3 * (a0 + j) + 1]);
                const float dz = __fsub_rn(zi, xyz[3 * (a0 + j) + 2]);
                const float d2 = __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
                // first guess from the distance, then exact comparisons with the squared edges
                // 1.25 + 0.5 k (k = 1..29), which are representable exactly
                int b = (int)((sqrtf(d2) - 1.25f) * 2.0f);
                b = b < 0 ? 0 : (b > kBins - 1 ? kBins - 1 : b);
                while (b < kBins - 1) {
                    const float e = 1.25f + 0.5f * (float)(b + 1);
                    if (d2 >= e * e) ++b; else break;
                }
                while (b > 0) {
                    const float e = 1.25f + 0.5f * (float)b;
                    if (d2 < e * e) --b; else break;
                }
                atomicAdd(&cnt[ti * kSlots + 1 + b], 1);
            }
        }
    }
    wave_sync();
    for (int f = lane; f < kRows * kSlots; f += kWave) {
        float v = 0.0f;
        if (ok) {
            const int c = (f % kSlots == kSlots - 1) ? d.B : cnt[f];
            v = log1pf((float)c);
            if (mean) v = (v - mean[f]) * istd[f];
        }
        if (out_f) out_f[(size_t)l * SURR_FEATURES + f] = v;
        if (out_b) out_b[(size_t)l * SURR_FEATURES + f] = f2bf(v);
    }
}

// Column statistics: FP64 partial sums per (chunk of rows, column), then a fixed-order total.
constexpr int kStatRows = 1024;

__global__ __launch_bounds__(64) void k_stats_partial(const float *__restrict__ F, int64_t n_rows,
                                                      double *__restrict__ part) {
    const int col = blockIdx.y * kWave + threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kStatRows, r1 = min(n_rows, r0 + kStatRows);
    double s = 0.0, q = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const double v = F[r * SURR_FEATURES + col];
        s += v;
        q += v * v;
    }
    part[((int64_t)blockIdx.x * SURR_FEATURES + col) * 2] = s;
    part[((int64_t)blockIdx.x * SURR_FEATURES + col) * 2 + 1] = q;
}

__global__ void k_stats_final(const double *__restrict__ part, int n_chunks, int64_t n_rows, float *mean,
                              float *istd) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= SURR_FEATURES) return;
    double s = 0.0, q = 0.0;
    for (int c = 0; c < n_chunks; ++c) {
        s += part[((int64_t)c * SURR_FEATURES + col) * 2];
        q += part[((int64_t)c * SURR_FEATURES + col) * 2 + 1];
    }
    const double m = s / (double)n_rows;
    const double var = fmax(q / (double)n_rows - m * m, 0.0);
    const double sd = sqrt(var);
    mean[col] = (float)m;
    istd[col] = sd < 1e-6 ? 1.0f : (float)(1.0 / sd);  // constant features are left unscaled
}

// ---------------------------------------------------------------------------------------------
// GEMM on the matrix cores: C = A B, BF16 operands, FP32 accumulation.
// A (m, k) is at A[m * lda + k] (A_K) or A[k * lda + m]; B (k, n) at B[n * ldb + k] (B_K) or
// B[k * ldb + n].  N is a multiple of 64 and K of 32; rows m >= M are skipped.
// Tiles of 64 x 64 per block of four wavefronts, each wavefront a 32 x 32 MFMA tile.
// ---------------------------------------------------------------------------------------------

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

enum { EPI_F32 = 0, EPI_BIAS_RELU_BF16 = 1, EPI_MASK_BF16 = 2, EPI_HEAD = 3 };

constexpr int kBM = 64, kBN = 64, kBK = 32, kPitch = kBK + 8;  // LDS rows padded against bank conflicts

template <bool A_K, bool B_K, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const uint16_t *__restrict__ A, int lda,
                                              const uint16_t *__restrict__ B, int ldb, float *__restrict__ Cf,
                                              uint16_t *__restrict__ Cb, int ldc, const float *__restrict__ bias,
                                              const uint16_t *__restrict__ mask, int ldm) {
    __shared__ __align__(16) uint16_t As[kBM * kPitch];
    __shared__ __align__(16) uint16_t Bs[kBN * kPitch];
    const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

    for (int k0 = 0; k0 < K; k0 += kBK) {
        // stage A and B tiles, K contiguous per row
        if constexpr (A_K) {
            const int r = t >> 2, c = (t & 3) * 8;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (m0 + r < M) v = *reinterpret_cast<const uint4 *>(A + (size_t)(m0 + r) * lda + k0 + c);
            *reinterpret_cast<uint4 *>(As + r * kPitch + c) = v;
        } else {
            const int kk = t >> 3, mm = (t & 7) * 8;
            uint16_t v[8];
            if (m0 + mm + 8 <= M) {
                const uint4 q = *reinterpret_cast<const uint4 *>(A + (size_t)(k0 + kk) * lda + m0 + mm);
                __builtin_memcpy(v, &q, 16);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = m0 + mm + i < M ? A[(size_t)(k0 + kk) * lda + m0 + mm + i] : 0;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) As[(mm + i) * kPitch + kk] = v[i];
        }
        if constexpr (B_K) {
            const int r = t >> 2, c = (t & 3) * 8;
            *reinterpret_cast<uint4 *>(Bs + r * kPitch + c) =
                *reinterpret_cast<const uint4 *>(B + (size_t)(n0 + r) * ldb + k0 + c);
        } else {
            const int kk = t >> 3, nn = (t & 7) * 8;
            const uint4 q = *reinterpret_cast<const uint4 *>(B + (size_t)(k0 + kk) * ldb + n0 + nn);
            uint16_t v[8];
            __builtin_memcpy(v, &q, 16);
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[(nn + i) * kPitch + kk] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 16) {
            const int kq = kk + 8 * (lane >> 5);
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(As + (wm * 32 + (lane & 31)) * kPitch + kq);
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(Bs + (wn * 32 + (lane & 31)) * kPitch + kq);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // lane holds column (lane & 31) of rows 8 (r / 4) + 4 (lane / 32) + r % 4 of its 32 x 32 tile
    const int col = n0 + wn * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row >= M) continue;
        const float v = acc[r];
        if constexpr (EPI == EPI_F32) {
            Cf[(size_t)row * ldc + col] = v;
        } else if constexpr (EPI == EPI_BIAS_RELU_BF16) {
            Cb[(size_t)row * ldc + col] = f2bf(fmaxf(v + bias[col], 0.0f));
        } else {
            Cb[(size_t)row * ldc + col] = bf2f(mask[(size_t)row * ldm + col]) > 0.0f ? f2bf(v) : (uint16_t)0;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Forward-layer GEMM, C = A B^T with A (M, K) and B (N, K) both K-contiguous (activations times
// weights): 128 x 128 tiles per block of four wavefronts, each wavefront a 64 x 64 tile of 2 x 2
// v_mfma_f32_32x32x16_bf16; K steps of 64 through two LDS buffers, the next step's operands loaded
// from global memory into registers while the current step's MFMAs run, one barrier per step.
// The MFMAs walk K in the same ascending 16-wide steps as k_gemm, so the results are identical.
// Tiles are numbered so that each XCD (blocks are dealt to the eight XCDs in turn) takes a
// contiguous run of them: the N tiles of one row block then run side by side in one L2.
// Requires N % 128 == 0 and K % 64 == 0; rows m >= M are skipped.
// Epilogues: EPI_BIAS_RELU_BF16 stores H = relu(C + bias) in BF16, staged through LDS so that
// the stores are 16-byte and row-contiguous.  EPI_HEAD (the last hidden layer at inference)
// stores nothing of H: each wavefront rounds its 64 x 64 tile of relu(C + bias) to BF16,
// multiplies it by the output weights w3 and sums each row over its 64 columns in a fixed order,
// writing part[row][2 (n tile) + wn]; k_head_sum adds the parts.
// ---------------------------------------------------------------------------------------------

constexpr int kTM = 128, kTN = 128, kTK = 64, kTP = kTK + 8;  // LDS pitch 144 B: conflict-free 16-B reads
constexpr int kXcds = 8;

template <int EPI>
__global__ __launch_bounds__(256, 2) void k_gemm_nt(int M, int N, int K, const uint16_t *__restrict__ A, int lda,
                                                    const uint16_t *__restrict__ B, int ldb,
                                                    uint16_t *__restrict__ Cb, int ldc,
                                                    const float *__restrict__ bias, const uint16_t *__restrict__ w3,
                                                    float *__restrict__ part) {
    // two A buffers then two B buffers; after the K loop the head epilogue reuses the space
    __shared__ __align__(16) uint16_t smem[4 * kTM * kTP];
    static_assert(4 * 64 * kTP <= 4 * kTM * kTP, "output staging tile does not fit");
    uint16_t(*As)[kTM * kTP] = reinterpret_cast<uint16_t(*)[kTM * kTP]>(smem);
    uint16_t(*Bs)[kTN * kTP] = reinterpret_cast<uint16_t(*)[kTN * kTP]>(smem + 2 * kTM * kTP);
    const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
    const int wm = w >> 1, wn = w & 1;
    const int ntn = N / kTN;
    const int nblk = (int)gridDim.x;
    int tile = (int)blockIdx.x;
    if (nblk % kXcds == 0) tile = (tile % kXcds) * (nblk / kXcds) + tile / kXcds;
    const int m0 = (tile / ntn) * kTM, n0 = (tile % ntn) * kTN;

    // global -> register staging: 128 rows x 64 k of A and of B in 16-byte chunks, four per thread
    // (chunk c = t + 256 i: row c / 8, k offset 8 (c % 8)).  Rows of A past M read row M - 1 and
    // are zeroed, so the loads carry no branch.
    const int lrow = t >> 3, lk = (t & 7) * 8;
    const uint16_t *ga[4], *gb[4];
    uint32_t live[4];  // all ones for rows inside M, zero past it
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = lrow + 32 * i;
        live[i] = m0 + row < M ? ~0u : 0u;
        ga[i] = A + (size_t)min(m0 + row, M - 1) * lda + lk;
        gb[i] = B + (size_t)(n0 + row) * ldb + lk;
    }
    auto masked = [](uint4 v, uint32_t mk) { return make_uint4(v.x & mk, v.y & mk, v.z & mk, v.w & mk); };
    const int lofs = lrow * kTP + lk;
    uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
#define LIGATE_GLOAD(k0)                                                              \
    do {                                                                              \
        ra0 = *reinterpret_cast<const uint4 *>(ga[0] + (k0));                        \
        ra1 = *reinterpret_cast<const uint4 *>(ga[1] + (k0));                        \
        ra2 = *reinterpret_cast<const uint4 *>(ga[2] + (k0));                        \
        ra3 = *reinterpret_cast<const uint4 *>(ga[3] + (k0));                        \
        rb0 = *reinterpret_cast<const uint4 *>(gb[0] + (k0));                        \
        rb1 = *reinterpret_cast<const uint4 *>(gb[1] + (k0));                        \
        rb2 = *reinterpret_cast<const uint4 *>(gb[2] + (k0));                        \
        rb3 = *reinterpret_cast<const uint4 *>(gb[3] + (k0));                        \
    } while (0)
#define LIGATE_LSTORE(buf)                                                            \
    do {                                                                              \
        *reinterpret_cast<uint4 *>(&As[buf][lofs]) = masked(ra0, live[0]);            \
        *reinterpret_cast<uint4 *>(&As[buf][lofs + 32 * kTP]) = masked(ra1, live[1]); \
        *reinterpret_cast<uint4 *>(&As[buf][lofs + 64 * kTP]) = masked(ra2, live[2]); \
        *reinterpret_cast<uint4 *>(&As[buf][lofs + 96 * kTP]) = masked(ra3, live[3]); \
        *reinterpret_cast<uint4 *>(&Bs[buf][lofs]) = rb0;                             \
        *reinterpret_cast<uint4 *>(&Bs[buf][lofs + 32 * kTP]) = rb1;                  \
        *reinterpret_cast<uint4 *>(&Bs[buf][lofs + 64 * kTP]) = rb2;                  \
        *reinterpret_cast<uint4 *>(&Bs[buf][lofs + 96 * kTP]) = rb3;                  \
    } while (0)

    f32x16 acc00, acc01, acc10, acc11;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc00[r] = acc01[r] = acc10[r] = acc11[r] = 0.0f;

    LIGATE_GLOAD(0);
    LIGATE_LSTORE(0);
    __syncthreads();
    const int nk = K / kTK;
    for (int ks = 0; ks < nk; ++ks) {
        const int cur = ks & 1;
        if (ks + 1 < nk) LIGATE_GLOAD((ks + 1) * kTK);  // in flight during this step's MFMAs
        const uint16_t *as = &As[cur][(wm * 64 + (lane & 31)) * kTP + 8 * (lane >> 5)];
        const uint16_t *bs = &Bs[cur][(wn * 64 + (lane & 31)) * kTP + 8 * (lane >> 5)];
#pragma unroll
        for (int kk = 0; kk < kTK; kk += 16) {
            const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(as + kk);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8 *>(as + 32 * kTP + kk);
            const bf16x8 b0 = *reinterpret_cast<const bf16x8 *>(bs + kk);
            const bf16x8 b1 = *reinterpret_cast<const bf16x8 *>(bs + 32 * kTP + kk);
            // operands swapped: each product is a 32 x 32 tile of C^T (the weights' rows first), so
            // a lane ends up holding four consecutive columns of one row of C
            acc00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b0, a0, acc00, 0, 0, 0);
            acc01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b1, a0, acc01, 0, 0, 0);
            acc10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b0, a1, acc10, 0, 0, 0);
            acc11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b1, a1, acc11, 0, 0, 0);
        }
        // the other buffer was last read in the previous step, before its closing barrier
        if (ks + 1 < nk) LIGATE_LSTORE(cur ^ 1);
        __syncthreads();
    }
#undef LIGATE_GLOAD
#undef LIGATE_LSTORE
    const f32x16 acc[2][2] = {{acc00, acc01}, {acc10, acc11}};
    // tile (i, j): lane holds row (lane & 31) of the i-th 32-row slice and, for q = 0..3, the columns
    // 8 q + 4 (lane / 32) + 0..3 of the j-th 32-column slice, in acc[i][j][4 q + 0..3]
    const int rl = lane & 31, ch = 4 * (lane >> 5);
    if constexpr (EPI == EPI_HEAD) {
        // each lane sums its 32 columns of a row (j, q, then the four columns), the two lanes that
        // share a row add their sums, lower half first
        float rs[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            float sum = 0.0f;
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int col = n0 + wn * 64 + j * 32 + 8 * q + ch + u;
                        sum += bf2f(f2bf(fmaxf(acc[i][j][4 * q + u] + bias[col], 0.0f))) * bf2f(w3[col]);
                    }
            const float other = __shfl_xor(sum, 32);
            rs[i] = lane < 32 ? sum + other : other + sum;
        }
        if (lane < 32) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = m0 + wm * 64 + i * 32 + rl;
                if (row < M) part[(size_t)row * (2 * ntn) + 2 * (tile % ntn) + wn] = rs[i];
            }
        }
    } else {
        // stage the wavefront's 64 x 64 BF16 tile in LDS (four columns per 8-byte write), then write
        // it out in 16-byte pieces, eight lanes per 128-byte row segment
        uint16_t *ct = smem + w * 64 * kTP;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int cl = j * 32 + 8 * q + ch, col = n0 + wn * 64 + cl;
                    uint32_t h[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) h[u] = f2bf(fmaxf(acc[i][j][4 * q + u] + bias[col + u], 0.0f));
                    *reinterpret_cast<uint2 *>(ct + (i * 32 + rl) * kTP + cl) =
                        make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
                }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = lane + 64 * k, r = c >> 3, q8 = (c & 7) * 8;
            const int row = m0 + wm * 64 + r;
            const uint4 v = *reinterpret_cast<const uint4 *>(ct + r * kTP + q8);
            if (row < M) *reinterpret_cast<uint4 *>(Cb + (size_t)row * ldc + n0 + wn * 64 + q8) = v;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Forward-layer GEMM for the network's own widths (K = 512 or 1024, N a multiple of BN), with the
// operands copied from global memory straight into LDS (global_load_lds_dwordx4: no register
// staging, no LDS store instructions) through a three-stage ring of K steps of 32, so that two K
// steps are in flight while a third is multiplied.
// * Block tile 128 x BN, four wavefronts of 64 x BN/2, each 2 x BN/64 v_mfma_f32_32x32x16_bf16
//   tiles, operands swapped as in k_gemm_nt (a lane holds four consecutive columns of one row).
//   The K order of every accumulator is that of k_gemm_nt, so the products are identical.
// * A stage holds the A rows then the B rows, 64 bytes each; 16-byte chunk c of row r sits in
//   slot c ^ ((r >> 2) & 3).  Measured on gfx950 (bank-conflict cycles per LDS instruction of the
//   whole kernel, epilogue included): no swizzle or r & 3: 9.5; (r >> 1) & 3 or ((r >> 1) ^ (r >> 3))
//   & 3: 3.4; (r >> 2) & 3, (r >> 3) & 3 or (r ^ (r >> 3)) & 3: 0.38.
//   Lane i of a copy instruction writes LDS bytes [16 i, 16 i + 16) of its 1 KB piece, so each
//   lane fetches the global chunk that belongs in that slot.
// * Each stage is a separate LDS array and the K loop is unrolled, so the compiler can tell the
//   copies into one stage from the fragment reads of another and adds no waits of its own; the
//   waits are explicit: before step k a wavefront waits until only its copies of step k + 1 are
//   outstanding, then all wavefronts meet at a barrier (after their LDS reads have completed,
//   since the copy issued next overwrites the stage read in the step before).
// * Rows of A past M load row M - 1 (finite values whose results are never stored).
// Epilogues as in k_gemm_nt: EPI_BIAS_RELU_BF16 stages relu(C + bias) in BF16 through LDS (two
// halves of 32 rows) for 16-byte row-contiguous stores; EPI_HEAD multiplies the BF16 tile by w3
// and writes per-row sums, part[row][2 (n tile) + wn], each over the wavefront's BN/2 columns.
// ---------------------------------------------------------------------------------------------

typedef __attribute__((address_space(3))) void lds_void;

// s_waitcnt vmcnt(n), leaving the other counters alone (n is a constant once the caller's loop is
// unrolled, so the switch folds to one instruction)
__device__ __forceinline__ void wait_vmcnt(int n) {
#define LIGATE_VMCNT(v) \
    case v: __builtin_amdgcn_s_waitcnt(((v) & 15) | (7 << 4) | (15 << 8) | (((v) >> 4) << 14)); break;
    switch (n) {
        LIGATE_VMCNT(0) LIGATE_VMCNT(1) LIGATE_VMCNT(2) LIGATE_VMCNT(3) LIGATE_VMCNT(4) LIGATE_VMCNT(5)
        LIGATE_VMCNT(6) LIGATE_VMCNT(7) LIGATE_VMCNT(8)
        default: __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8)); break;
    }
#undef LIGATE_VMCNT
}

__device__ __forceinline__ int ring_swizzle(int r) { return (r >> 2) & 3; }

constexpr int kRingBK = 32, kRingStages = 3;

template <int EPI, int BN, int NK>
__global__ __launch_bounds__(256, BN == 128 ? 3 : 2) void k_gemm_lds(int M, int N, const uint16_t *__restrict__ A,
                                                                     const uint16_t *__restrict__ B,
                                                                     uint16_t *__restrict__ Cb,
                                                                     const float *__restrict__ bias,
                                                                     const uint16_t *__restrict__ w3,
                                                                     float *__restrict__ part) {
    constexpr int BK = kRingBK, NS = kRingStages, CH = BK / 8;
    constexpr int STAGE = (kTM + BN) * BK;      // BF16 values per stage
    constexpr int WN = BN / 2, NJ = WN / 32;    // columns per wavefront, 32-wide MFMA tiles along them
    constexpr int LA = kTM * CH / 256, LB = BN * CH / 256, LPW = LA + LB;  // copies per wavefront per stage
    constexpr int K = NK * BK;
    static_assert(2 * 32 * WN <= STAGE, "output staging does not fit a stage");
    __shared__ __align__(16) uint16_t s0[STAGE];
    __shared__ __align__(16) uint16_t s1[STAGE];
    __shared__ __align__(16) uint16_t s2[STAGE];
    __shared__ __align__(16) float sbias[BN];
    __shared__ __align__(16) uint16_t sw3[EPI == EPI_HEAD ? BN : 8];
    uint16_t *const stg[NS] = {s0, s1, s2};
    const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
    const int wm = w >> 1, wn = w & 1;
    const int ntn = N / BN;
    const int nblk = (int)gridDim.x;
    int tile = (int)blockIdx.x;
    if (nblk % kXcds == 0) tile = (tile % kXcds) * (nblk / kXcds) + tile / kXcds;
    const int m0 = (tile / ntn) * kTM, n0 = (tile % ntn) * BN;

    // the global chunk each lane copies, per copy instruction: piece p = w L + q of the A (B) rows
    const uint16_t *ga[LA], *gb[LB];
#pragma unroll
    for (int q = 0; q < LA; ++q) {
        const int P = (w * LA + q) * kWave + lane, r = P / CH, c = (P % CH) ^ ring_swizzle(r);
        ga[q] = A + (size_t)min(m0 + r, M - 1) * K + c * 8;
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
        const int P = (w * LB + q) * kWave + lane, r = P / CH, c = (P % CH) ^ ring_swizzle(r);
        gb[q] = B + (size_t)(n0 + r) * K + c * 8;
    }
    auto issue = [&](int ks, int buf) {
        uint16_t *base = stg[buf];
#pragma unroll
        for (int q = 0; q < LA; ++q)
            __builtin_amdgcn_global_load_lds((const void *)(ga[q] + ks * BK), (lds_void *)(base + (w * LA + q) * 512),
                                             16, 0, 0);
#pragma unroll
        for (int q = 0; q < LB; ++q)
            __builtin_amdgcn_global_load_lds((const void *)(gb[q] + ks * BK),
                                             (lds_void *)(base + kTM * BK + (w * LB + q) * 512), 16, 0, 0);
    };

    f32x16 acc[2][NJ];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    // bias (and the BF16 w3) of the tile's columns, copied into LDS ahead of the ring's first stages
    // (so the waits for those stages cover them too) and read after the ring's first barrier
    if (w < BN / kWave)
        __builtin_amdgcn_global_load_lds((const void *)(bias + n0 + kWave * w + lane), (lds_void *)(sbias + kWave * w),
                                         4, 0, 0);
    if constexpr (EPI == EPI_HEAD) {
        if (w < BN / (2 * kWave))  // pairs of BF16 values as 4-byte words
            __builtin_amdgcn_global_load_lds((const void *)(reinterpret_cast<const uint32_t *>(w3 + n0) + kWave * w + lane),
                                             (lds_void *)(sw3 + 2 * kWave * w), 4, 0, 0);
    }
#pragma unroll
    for (int s = 0; s < NS - 1; ++s) issue(s, s);
    const int fl = ring_swizzle(lane & 31);  // rows read by this lane differ by multiples of 32
    const int arow = (wm * 64 + (lane & 31)) * BK, brow = kTM * BK + (wn * WN + (lane & 31)) * BK;
#pragma unroll
    for (int ks0 = 0; ks0 < NK; ks0 += NS) {
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            const int ks = ks0 + st;
            if (ks >= NK) break;
            const int ahead = NK - 1 - ks;  // copies of later steps already issued: min(ahead, NS - 2) steps
            wait_vmcnt(LPW * (ahead < NS - 2 ? ahead : NS - 2));
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
            if (ks + NS - 1 < NK) issue(ks + NS - 1, (st + NS - 1) % NS);
            const uint16_t *S = stg[st];
#pragma unroll
            for (int kk = 0; kk < BK; kk += 16) {
                const int off = (((kk >> 3) + (lane >> 5)) ^ fl) << 3;
                bf16x8 a[2], b[NJ];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(S + arow + i * 32 * BK + off);
#pragma unroll
                for (int j = 0; j < NJ; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(S + brow + j * 32 * BK + off);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[j], a[i], acc[i][j], 0, 0, 0);
            }
        }
    }
    // tile (i, j): lane holds row i 32 + (lane & 31) and, for q = 0..3, the columns j 32 + 8 q +
    // 4 (lane / 32) + 0..3 of the wavefront's columns, in acc[i][j][4 q + 0..3]
    const int rl = lane & 31, ch = 4 * (lane >> 5);
    if constexpr (EPI == EPI_HEAD) {
        // each lane sums its columns of a row (j, q, then the four columns), the two lanes that share
        // a row add their sums, lower half first
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            float sum = 0.0f;
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int cl = wn * WN + j * 32 + 8 * q + ch;
                    const float4 bb = *reinterpret_cast<const float4 *>(sbias + cl);
                    const uint2 ww = *reinterpret_cast<const uint2 *>(sw3 + cl);
                    sum += bf2f(f2bf(fmaxf(acc[i][j][4 * q + 0] + bb.x, 0.0f))) * bf2f((uint16_t)ww.x);
                    sum += bf2f(f2bf(fmaxf(acc[i][j][4 * q + 1] + bb.y, 0.0f))) * bf2f((uint16_t)(ww.x >> 16));
                    sum += bf2f(f2bf(fmaxf(acc[i][j][4 * q + 2] + bb.z, 0.0f))) * bf2f((uint16_t)ww.y);
                    sum += bf2f(f2bf(fmaxf(acc[i][j][4 * q + 3] + bb.w, 0.0f))) * bf2f((uint16_t)(ww.y >> 16));
                }
            const float other = __shfl_xor(sum, 32);
            const float rs = lane < 32 ? sum + other : other + sum;
            const int row = m0 + wm * 64 + i * 32 + rl;
            if (lane < 32 && row < M) part[(size_t)row * (2 * ntn) + 2 * (tile % ntn) + wn] = rs;
        }
    } else {
        // per half i: each wavefront stages its 32 x WN BF16 tile (rows of 2 WN bytes, 16-byte chunk c
        // of row r in slot c ^ (r & 7)) in s0 (wavefronts 0, 1) or s1 (2, 3), then stores it in
        // 16-byte row-contiguous pieces
        constexpr int RC = WN / 8;
        wait_vmcnt(0);
        __syncthreads();  // the ring is no longer read
        uint16_t *ct = (w < 2 ? s0 : s1) + (w & 1) * 32 * WN;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int cl = j * 32 + 8 * q + ch;
                    const float4 bb = *reinterpret_cast<const float4 *>(sbias + wn * WN + cl);
                    const uint32_t h0 = f2bf(fmaxf(acc[i][j][4 * q + 0] + bb.x, 0.0f));
                    const uint32_t h1 = f2bf(fmaxf(acc[i][j][4 * q + 1] + bb.y, 0.0f));
                    const uint32_t h2 = f2bf(fmaxf(acc[i][j][4 * q + 2] + bb.z, 0.0f));
                    const uint32_t h3 = f2bf(fmaxf(acc[i][j][4 * q + 3] + bb.w, 0.0f));
                    *reinterpret_cast<uint2 *>(ct + rl * WN + (((cl >> 3) ^ (rl & 7)) << 3) + ch) =
                        make_uint2(h0 | (h1 << 16), h2 | (h3 << 16));
                }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < RC / 2; ++k) {
                const int c = lane + kWave * k, r = c / RC, cc = c % RC;
                const int row = m0 + wm * 64 + i * 32 + r;
                const uint4 v = *reinterpret_cast<const uint4 *>(ct + r * WN + ((cc ^ (r & 7)) << 3));
                if (row < M) *reinterpret_cast<uint4 *>(Cb + (size_t)row * N + n0 + wn * WN + cc * 8) = v;
            }
            __syncthreads();
        }
    }
}

// y[row] = (sum of the row's parts in order) + b3.
__global__ void k_head_sum(const float *__restrict__ part, int n_part, int M, const float *__restrict__ b3,
                           float *__restrict__ y) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= M) return;
    float s = 0.0f;
    for (int q = 0; q < n_part; ++q) s += part[(size_t)row * n_part + q];
    y[row] = s + b3[0];
}

template <bool A_K, bool B_K, int EPI>
static void gemm(hipStream_t st, int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B, int ldb,
                 float *Cf, uint16_t *Cb, int ldc, const float *bias = nullptr, const uint16_t *mask = nullptr,
                 int ldm = 0) {
    dim3 grid((unsigned)(N / kBN), (unsigned)((M + kBM - 1) / kBM));
    hipLaunchKernelGGL((k_gemm<A_K, B_K, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, Cf, Cb, ldc, bias,
                       mask, ldm);
}

// ---------------------------------------------------------------------------------------------
// Output layer, loss, reductions, Adam
// ---------------------------------------------------------------------------------------------

// y[b] = sum_k H2[b][k] w3[k] + b3; with targets also r2[b] = (y - t)^2 and dy[b] = 2 (y - t) / B.
__global__ __launch_bounds__(64) void k_head(const uint16_t *__restrict__ H2, int h2, const uint16_t *__restrict__ w3,
                                             const float *__restrict__ b3, int batch, float *__restrict__ y,
                                             const float *__restrict__ target, float *__restrict__ r2,
                                             float *__restrict__ dy) {
    const int b = blockIdx.x, lane = lane_id();
    float acc = 0.0f;
    for (int k = lane; k < h2; k += kWave) acc = fmaf(bf2f(H2[(size_t)b * h2 + k]), bf2f(w3[k]), acc);
    const float v = wave_sum(acc) + b3[0];
    if (lane == 0) {
        if (y) y[b] = v;
        if (target) {
            const float e = v - target[b];
            r2[b] = e * e;
            dy[b] = 2.0f * e / (float)batch;
        }
    }
}

// loss = sum r2 / B and db3 = sum dy, in a fixed order (one wavefront).
__global__ __launch_bounds__(64) void k_loss(const float *__restrict__ r2, const float *__restrict__ dy, int batch,
                                             float *loss, float *db3) {
    const int lane = lane_id();
    float s = 0.0f, g = 0.0f;
    for (int b = lane; b < batch; b += kWave) {
        s += r2[b];
        g += dy[b];
    }
    s = wave_sum(s);
    g = wave_sum(g);
    if (lane == 0) {
        *loss = s / (float)batch;
        *db3 = g;
    }
}

// dH2[b][k] = dy[b] w3[k] where H2[b][k] > 0, stored in BF16.
__global__ void k_head_back(const uint16_t *__restrict__ H2, const uint16_t *__restrict__ w3,
                            const float *__restrict__ dy, int batch, int h2, uint16_t *__restrict__ dH2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)batch * h2) return;
    const int b = (int)(i / h2), k = (int)(i - (int64_t)b * h2);
    dH2[i] = bf2f(H2[i]) > 0.0f ? f2bf(dy[b] * bf2f(w3[k])) : (uint16_t)0;
}

// out[c] = sum_r wgt[r] X[r][c] (wgt == NULL: plain sum).  A block takes 64 columns; its four
// wavefronts take the rows r = g, g + 4, g + 8, ... (g = wavefront), each in order, and the four
// partial sums are added in wavefront order: a fixed order, with coalesced 128-byte row reads.
constexpr int kColGroups = 4;
__global__ __launch_bounds__(kWave *kColGroups) void k_colsum(const uint16_t *__restrict__ X, int rows, int cols,
                                                             const float *__restrict__ wgt,
                                                             float *__restrict__ out) {
    __shared__ float part[kColGroups][kWave];
    const int g = threadIdx.x / kWave, lane = lane_id(), c = blockIdx.x * kWave + lane;
    float s = 0.0f;
    if (c < cols) {
        for (int r = g; r < rows; r += kColGroups) {
            const float v = bf2f(X[(size_t)r * cols + c]);
            s = wgt ? fmaf(wgt[r], v, s) : s + v;
        }
    }
    part[g][lane] = s;
    __syncthreads();
    if (g == 0 && c < cols) {
        float t = part[0][lane];
        for (int q = 1; q < kColGroups; ++q) t += part[q][lane];
        out[c] = t;
    }
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// BF16 copies of W1, W2 and w3 from the master weights.
__global__ void k_cast(const float *__restrict__ master, uint16_t *__restrict__ out, int64_t n_w1, int64_t off_w2,
                       int64_t n_w2, int64_t off_w3, int64_t n_w3) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_w1) out[i] = f2bf(master[i]);
    else if (i < n_w1 + n_w2) out[i] = f2bf(master[off_w2 + (i - n_w1)]);
    else if (i < n_w1 + n_w2 + n_w3) out[i] = f2bf(master[off_w3 + (i - n_w1 - n_w2)]);
}

// ---------------------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------------------

struct Layout {  // offsets into the master / BF16 arrays
    int64_t W1, b1, W2, b2, w3, b3, n_master;
    int64_t bW1, bW2, bw3, n_bf16;
    static Layout of(int d, int h1, int h2) {
        Layout L;
        L.W1 = 0;
        L.b1 = L.W1 + (int64_t)h1 * d;
        L.W2 = L.b1 + h1;
        L.b2 = L.W2 + (int64_t)h2 * h1;
        L.w3 = L.b2 + h2;
        L.b3 = L.w3 + h2;
        L.n_master = L.b3 + 1;
        L.bW1 = 0;
        L.bW2 = (int64_t)h1 * d;
        L.bw3 = L.bW2 + (int64_t)h2 * h1;
        L.n_bf16 = L.bw3 + h2;
        return L;
    }
};

static size_t al(size_t v) { return (v + 255) & ~size_t(255); }

static int check_model(const surr_model *m, bool need_train) {
    LIGATE_REQUIRE(m != nullptr, DOCK_ERR_INVALID_ARG, "model is NULL");
    LIGATE_REQUIRE(m->d_in > 0 && m->h1 > 0 && m->h2 > 0 && m->d_in % 64 == 0 && m->h1 % 64 == 0 && m->h2 % 64 == 0,
                   DOCK_ERR_INVALID_ARG, "layer widths must be positive multiples of 64");
    LIGATE_REQUIRE(m->d_master && m->d_bf16, DOCK_ERR_INVALID_ARG, "model weights are NULL");
    if (need_train)
        LIGATE_REQUIRE(m->d_grad && m->d_adam_m && m->d_adam_v, DOCK_ERR_INVALID_ARG, "training buffers are NULL");
    return DOCK_OK;
}

struct FwdWs {
    uint16_t *H1, *H2;
};

static size_t fwd_ws_bytes(const surr_model *m, int batch) {
    return al(2 * (size_t)batch * m->h1) + al(2 * (size_t)batch * m->h2);
}

static FwdWs fwd_ws(const surr_model *m, int batch, void *ws) {
    char *p = (char *)ws;
    FwdWs w;
    w.H1 = (uint16_t *)p;
    w.H2 = (uint16_t *)(p + al(2 * (size_t)batch * m->h1));
    return w;
}

// A forward layer: H = relu(X W^T + b) in BF16, on the large-tile kernel where the shape allows.
static unsigned lds_tiles(int M, int N, int BN) { return (unsigned)((int64_t)((M + kTM - 1) / kTM) * (N / BN)); }

static void forward_layer(hipStream_t st, int M, int N, int K, const uint16_t *X, const uint16_t *W, uint16_t *H,
                          const float *bias) {
    const uint16_t *no_w3 = nullptr;
    float *no_part = nullptr;
    if (N % 128 == 0 && K == 512) {
        hipLaunchKernelGGL((k_gemm_lds<EPI_BIAS_RELU_BF16, 128, 16>), dim3(lds_tiles(M, N, 128)), dim3(256), 0, st, M,
                           N, X, W, H, bias, no_w3, no_part);
    } else if (N % 128 == 0 && K == 1024) {
        hipLaunchKernelGGL((k_gemm_lds<EPI_BIAS_RELU_BF16, 128, 32>), dim3(lds_tiles(M, N, 128)), dim3(256), 0, st, M,
                           N, X, W, H, bias, no_w3, no_part);
    } else if (N % kTN == 0 && K % kTK == 0) {
        const int64_t tiles = (int64_t)((M + kTM - 1) / kTM) * (N / kTN);
        hipLaunchKernelGGL((k_gemm_nt<EPI_BIAS_RELU_BF16>), dim3((unsigned)tiles), dim3(256), 0, st, M, N, K, X, K, W,
                           K, H, N, bias, (const uint16_t *)nullptr, (float *)nullptr);
    } else {
        gemm<true, true, EPI_BIAS_RELU_BF16>(st, M, N, K, X, K, W, K, nullptr, H, N, bias);
    }
}

static void run_forward(const surr_model *m, const Layout &L, const uint16_t *x, int batch, const FwdWs &w,
                        hipStream_t st) {
    forward_layer(st, batch, m->h1, m->d_in, x, m->d_bf16 + L.bW1, w.H1, m->d_master + L.b1);
    forward_layer(st, batch, m->h2, m->h1, w.H1, m->d_bf16 + L.bW2, w.H2, m->d_master + L.b2);
}

}  // namespace ligate

using namespace ligate;

extern "C" int surr_param_count(int32_t d_in, int32_t h1, int32_t h2, int64_t *n_master, int64_t *n_bf16) {
    LIGATE_ABI_RANGE();
    LIGATE_REQUIRE(d_in > 0 && h1 > 0 && h2 > 0 && n_master && n_bf16, DOCK_ERR_INVALID_ARG, "bad widths");
    const Layout L = Layout::of(d_in, h1, h2);
    *n_master = L.n_master;
    *n_bf16 = L.n_bf16;
    return DOCK_OK;
}

extern "C" int surr_features(const int32_t *d_atom_off, const float *d_xyz, const uint8_t *d_type, const void *d_pack,
                             int32_t n_lig, int64_t n_atoms_total, int32_t n_types, const float *d_mean,
                             const float *d_istd, float *d_feat, uint16_t *d_feat_bf16, void *stream) {
    LIGATE_ABI_RANGE();
    LIGATE_REQUIRE(n_lig >= 0 && n_atoms_total >= 0 && n_atoms_total < (1ll << 31), DOCK_ERR_INVALID_ARG,
                   "bad library size");
    LIGATE_REQUIRE(n_types >= 1 && n_types <= SURR_MAX_TYPES, DOCK_ERR_LIMIT, "features need n_types <= 16");
    LIGATE_REQUIRE((d_mean == nullptr) == (d_istd == nullptr), DOCK_ERR_INVALID_ARG, "mean and istd go together");
    LIGATE_REQUIRE(d_feat || d_feat_bf16, DOCK_ERR_INVALID_ARG, "no output");
    if (n_lig == 0) return DOCK_OK;
    LIGATE_REQUIRE(d_atom_off && d_xyz && d_type && d_pack, DOCK_ERR_INVALID_ARG, "NULL input");
    const PackView pk = PackView::of(d_pack, n_lig, n_atoms_total);
    hipLaunchKernelGGL(k_features, dim3((unsigned)n_lig), dim3(kWave), 0, (hipStream_t)stream, d_atom_off, d_xyz,
                       d_type, pk, d_mean, d_istd, d_feat, d_feat_bf16);
    return check_launch("surr_features");
}

extern "C" int surr_feature_stats(const float *d_feat, int64_t n_rows, float *d_mean, float *d_istd, void *d_ws,
                                  size_t *ws_bytes, void *stream) {
    LIGATE_ABI_RANGE();
    LIGATE_REQUIRE(n_rows >= 1 && ws_bytes, DOCK_ERR_INVALID_ARG, "bad arguments");
    const int64_t chunks = (n_rows + kStatRows - 1) / kStatRows;
    const size_t need = al(sizeof(double) * 2 * SURR_FEATURES * (size_t)chunks);
    if (d_ws == nullptr) {
        *ws_bytes = need;
        return DOCK_OK;
    }
    LIGATE_REQUIRE(*ws_bytes >= need, DOCK_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", *ws_bytes, need);
    LIGATE_REQUIRE(d_feat && d_mean && d_istd, DOCK_ERR_INVALID_ARG, "NULL array");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_stats_partial, dim3((unsigned)chunks, SURR_FEATURES / kWave), dim3(kWave), 0, st, d_feat,
                       n_rows, (double *)d_ws);
    hipLaunchKernelGGL(k_stats_final, dim3(SURR_FEATURES / 256), dim3(256), 0, st, (const double *)d_ws, (int)chunks,
                       n_rows, d_mean, d_istd);
    return check_launch("surr_feature_stats");
}

extern "C" int surr_cast(const surr_model *m, void *stream) {
    LIGATE_ABI_RANGE();
    int rc = check_model(m, false);
    if (rc) return rc;
    const Layout L = Layout::of(m->d_in, m->h1, m->h2);
    const int64_t n = L.n_bf16;
    hipLaunchKernelGGL(k_cast, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, m->d_master,
                       m->d_bf16, (int64_t)m->h1 * m->d_in, L.W2, (int64_t)m->h2 * m->h1, L.w3, (int64_t)m->h2);
    return check_launch("surr_cast");
}

extern "C" int surr_forward(const surr_model *m, const uint16_t *d_x, int32_t batch, float *d_y, void *d_ws,
                            size_t *ws_bytes, void *stream) {
    LIGATE_ABI_RANGE();
    int rc = check_model(m, false);
    if (rc) return rc;
    LIGATE_REQUIRE(batch >= 1 && ws_bytes, DOCK_ERR_INVALID_ARG, "bad batch");
    const size_t need = fwd_ws_bytes(m, batch);
    if (d_ws == nullptr) {
        *ws_bytes = need;
        return DOCK_OK;
    }
    LIGATE_REQUIRE(*ws_bytes >= need, DOCK_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", *ws_bytes, need);
    LIGATE_REQUIRE(d_x && d_y, DOCK_ERR_INVALID_ARG, "NULL array");
    hipStream_t st = (hipStream_t)stream;
    const Layout L = Layout::of(m->d_in, m->h1, m->h2);
    const FwdWs w = fwd_ws(m, batch, d_ws);
    if (m->h2 % kTN == 0 && m->h1 % kTK == 0) {
        // inference: the output layer is fused into the last hidden layer's epilogue (H2 is never
        // stored; the per-tile row sums go where H2 would be, at most 2 h2 / 128 floats per row)
        forward_layer(st, batch, m->h1, m->d_in, d_x, m->d_bf16 + L.bW1, w.H1, m->d_master + L.b1);
        float *part = reinterpret_cast<float *>(w.H2);
        int n_part;
        if (m->h2 % 256 == 0 && m->h1 == 1024) {
            n_part = 2 * (m->h2 / 256);
            hipLaunchKernelGGL((k_gemm_lds<EPI_HEAD, 256, 32>), dim3(lds_tiles(batch, m->h2, 256)), dim3(256), 0, st,
                               batch, m->h2, w.H1, m->d_bf16 + L.bW2, (uint16_t *)nullptr, m->d_master + L.b2,
                               m->d_bf16 + L.bw3, part);
        } else {
            n_part = 2 * (m->h2 / kTN);
            const int64_t tiles = (int64_t)((batch + kTM - 1) / kTM) * (m->h2 / kTN);
            hipLaunchKernelGGL((k_gemm_nt<EPI_HEAD>), dim3((unsigned)tiles), dim3(256), 0, st, batch, m->h2, m->h1,
                               w.H1, m->h1, m->d_bf16 + L.bW2, m->h1, (uint16_t *)nullptr, 0, m->d_master + L.b2,
                               m->d_bf16 + L.bw3, part);
        }
        hipLaunchKernelGGL(k_head_sum, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, st, part, n_part, batch,
                           m->d_master + L.b3, d_y);
    } else {
        run_forward(m, L, d_x, batch, w, st);
        hipLaunchKernelGGL(k_head, dim3((unsigned)batch), dim3(kWave), 0, st, w.H2, m->h2, m->d_bf16 + L.bw3,
                           m->d_master + L.b3, batch, d_y, (const float *)nullptr, (float *)nullptr, (float *)nullptr);
    }
    return check_launch("surr_forward");
}

extern "C" int surr_backward(const surr_model *m, const uint16_t *d_x, const float *d_t, int32_t batch, float *d_loss,
                             void *d_ws, size_t *ws_bytes, void *stream) {
    LIGATE_ABI_RANGE();
    int rc = check_model(m, true);
    if (rc) return rc;
    LIGATE_REQUIRE(batch >= 32 && batch % 32 == 0 && ws_bytes, DOCK_ERR_INVALID_ARG,
                   "batch must be a positive multiple of 32");
    const size_t f = fwd_ws_bytes(m, batch);
    const size_t need = f + al(2 * (size_t)batch * m->h2) + al(2 * (size_t)batch * m->h1) + 2 * al(4 * (size_t)batch);
    if (d_ws == nullptr) {
        *ws_bytes = need;
        return DOCK_OK;
    }
    LIGATE_REQUIRE(*ws_bytes >= need, DOCK_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", *ws_bytes, need);
    LIGATE_REQUIRE(d_x && d_t && d_loss, DOCK_ERR_INVALID_ARG, "NULL array");
    hipStream_t st = (hipStream_t)stream;
    const Layout L = Layout::of(m->d_in, m->h1, m->h2);
    const FwdWs w = fwd_ws(m, batch, d_ws);
    char *p = (char *)d_ws + f;
    uint16_t *dH2 = (uint16_t *)p;
    p += al(2 * (size_t)batch * m->h2);
    uint16_t *dH1 = (uint16_t *)p;
    p += al(2 * (size_t)batch * m->h1);
    float *dy = (float *)p;
    p += al(4 * (size_t)batch);
    float *r2 = (float *)p;
    float *g = m->d_grad;

    run_forward(m, L, d_x, batch, w, st);
    hipLaunchKernelGGL(k_head, dim3((unsigned)batch), dim3(kWave), 0, st, w.H2, m->h2, m->d_bf16 + L.bw3,
                       m->d_master + L.b3, batch, (float *)nullptr, d_t, r2, dy);
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(kWave), 0, st, r2, dy, batch, d_loss, g + L.b3);
    // output layer
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((m->h2 + kWave - 1) / kWave)), dim3(kWave * kColGroups), 0, st, w.H2, batch, m->h2, dy,
                       g + L.w3);
    const int64_t n2 = (int64_t)batch * m->h2;
    hipLaunchKernelGGL(k_head_back, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, w.H2, m->d_bf16 + L.bw3, dy,
                       batch, m->h2, dH2);
    // second layer: dW2 = dH2^T H1, db2 = column sums of dH2, dH1 = (dH2 W2) where H1 > 0
    gemm<false, false, EPI_F32>(st, m->h2, m->h1, batch, dH2, m->h2, w.H1, m->h1, g + L.W2, nullptr, m->h1);
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((m->h2 + kWave - 1) / kWave)), dim3(kWave * kColGroups), 0, st, dH2, batch, m->h2,
                       (const float *)nullptr, g + L.b2);
    gemm<true, false, EPI_MASK_BF16>(st, batch, m->h1, m->h2, dH2, m->h2, m->d_bf16 + L.bW2, m->h1, nullptr, dH1,
                                     m->h1, nullptr, w.H1, m->h1);
    // first layer: dW1 = dH1^T x, db1 = column sums of dH1
    gemm<false, false, EPI_F32>(st, m->h1, m->d_in, batch, dH1, m->h1, d_x, m->d_in, g + L.W1, nullptr, m->d_in);
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((m->h1 + kWave - 1) / kWave)), dim3(kWave * kColGroups), 0, st, dH1, batch, m->h1,
                       (const float *)nullptr, g + L.b1);
    return check_launch("surr_backward");
}

extern "C" int surr_adam(const surr_model *m, float lr, float beta1, float beta2, float eps, int32_t step,
                         void *stream) {
    LIGATE_ABI_RANGE();
    int rc = check_model(m, true);
    if (rc) return rc;
    LIGATE_REQUIRE(step >= 1 && lr > 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f &&
                       eps > 0.0f,
                   DOCK_ERR_INVALID_ARG, "bad Adam hyper-parameters");
    const Layout L = Layout::of(m->d_in, m->h1, m->h2);
    const double c1 = 1.0 / (1.0 - pow((double)beta1, (double)step));
    const double c2 = 1.0 / (1.0 - pow((double)beta2, (double)step));
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((L.n_master + 255) / 256)), dim3(256), 0, st, m->d_master, m->d_grad,
                       m->d_adam_m, m->d_adam_v, L.n_master, lr, beta1, beta2, eps, (float)c1, (float)c2);
    rc = check_launch("surr_adam");
    if (rc) return rc;
    return surr_cast(m, stream);
}

namespace ligate {
__global__ void k_gather_rows(const uint16_t *__restrict__ src, const int32_t *__restrict__ idx, int64_t n_idx,
                              int row, uint16_t *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_idx * row) return;
    const int64_t r = i / row;
    dst[i] = src[(int64_t)idx[r] * row + (i - r * row)];
}
__global__ void k_gather_f32(const float *__restrict__ src, const int32_t *__restrict__ idx, int64_t n_idx,
                             float *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_idx) dst[i] = src[idx[i]];
}
}  // namespace ligate

extern "C" int surr_gather(const uint16_t *d_x, const float *d_t, const int32_t *d_idx, int64_t n_idx, int32_t row,
                           uint16_t *d_x_out, float *d_t_out, void *stream) {
    LIGATE_ABI_RANGE();
    LIGATE_REQUIRE(n_idx >= 0 && row >= 1 && d_idx, DOCK_ERR_INVALID_ARG, "bad gather arguments");
    LIGATE_REQUIRE((d_x == nullptr) == (d_x_out == nullptr) && (d_t == nullptr) == (d_t_out == nullptr),
                   DOCK_ERR_INVALID_ARG, "inputs and outputs go together");
    if (n_idx == 0) return DOCK_OK;
    hipStream_t st = (hipStream_t)stream;
    if (d_x) {
        const int64_t n = n_idx * row;
        hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d_x, d_idx, n_idx, row,
                           d_x_out);
    }
    if (d_t)
        hipLaunchKernelGGL(k_gather_f32, dim3((unsigned)((n_idx + 255) / 256)), dim3(256), 0, st, d_t, d_idx, n_idx,
                           d_t_out);
    return check_launch("surr_gather");
}

namespace ligate {
__global__ void k_average(const float *__restrict__ y, int n_members, int64_t n, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int m = 0; m < n_members; ++m) s += y[(int64_t)m * n + i];
    out[i] = s / (float)n_members;
}
}  // namespace ligate

extern "C" int surr_average(const float *d_y, int32_t n_members, int64_t n, float *d_out, void *stream) {
    LIGATE_ABI_RANGE();
    LIGATE_REQUIRE(n_members >= 1 && n_members <= 64 && n >= 0, DOCK_ERR_INVALID_ARG, "bad ensemble size");
    if (n == 0) return DOCK_OK;
    LIGATE_REQUIRE(d_y && d_out, DOCK_ERR_INVALID_ARG, "NULL array");
    hipLaunchKernelGGL(k_average, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, d_y,
                       n_members, n, d_out);
    return check_launch("surr_average");
}
