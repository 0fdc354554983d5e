// Leaf value network on gfx950: a ReLU MLP evaluated and trained with
// bfloat16 MFMA GEMMs that accumulate in FP32 (v_mfma_f32_32x32x16_bf16).
//
// The paper evaluates every depth-limit leaf of an iteration in one batched
// forward pass (Sec. 4.3, Stage 5) of a network of the players' normalised
// reach probabilities and the public state (Sec. 3, the depth-limited solving
// equation); it trains that network as prior work does (Sec. 2) without
// giving an architecture.  Here: d_in -> width x depth (ReLU) -> d_out,
// weights kept as FP32 masters with bfloat16 copies for the GEMMs, trained
// with a Huber loss and Adam.
//
// Every GEMM has the form C[M,N] = A[M,K] * B[N,K]^T with both operands
// K-contiguous; the backward pass forms the transposed operands it needs with
// a tiled transpose kernel.  All dimensions are padded to multiples of 64 and
// padding entries are zero.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "host.hpp"
#include "leafnet.hpp"

namespace pcfr {

typedef __attribute__((ext_vector_type(8))) __bf16 v8bf;
typedef __attribute__((ext_vector_type(16))) float v16f;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;   // 16-byte copies kept in registers

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------------ GEMM
// Workgroup tile BM x BN, 4 waves in a 2 x 2 grid, each wave (BM/2) x (BN/2)
// made of 32 x 32 MFMA tiles; K staged through LDS 64 at a time, double
// buffered, rows padded by 8 elements against bank conflicts.
//   EPI_BIAS_F32      C = A B^T + bias           (float out)
//   EPI_BIAS_RELU_BF  C = relu(A B^T + bias)     (bf16 out)
//   EPI_F32           C = A B^T                  (float out)
//   EPI_MASK_BF       C = (A B^T) * [mask > 0]   (bf16 out, mask bf16 [M][ldc])
//   EPI_BIAS_RELU_SWZ C = relu(A B^T + bias)     (bf16 out, in the swizzled layout below)
enum { EPI_BIAS_F32 = 0, EPI_BIAS_RELU_BF = 1, EPI_F32 = 2, EPI_MASK_BF = 3, EPI_BIAS_RELU_SWZ = 4 };

// Swizzled bf16 layout of an [R][K] matrix (R a multiple of 32, K of 16),
// for operands read straight into MFMA registers: the 16-byte chunk of row r
// holding columns [8q, 8q + 8) is chunk (r % 32) + 32 (q % 2) of block
// (r / 32, q / 2); blocks of 64 chunks are ordered by row block, then column
// block.  One A or B operand of v_mfma_f32_32x32x16_bf16 (32 rows x 16 K
// values) is then one block: 1 KB, lane l reading chunk l.
__host__ __device__ __forceinline__ int64_t swz_index(int64_t r, int64_t k, int64_t K) {
    return ((((r >> 5) * (K >> 4) + (k >> 4)) * 64) + (r & 31) + 32 * ((k >> 3) & 1)) * 8 + (k & 7);
}

// Output tile of workgroup `lin` of a 1-D grid over an mt x nt tile grid.
// Workgroups are dispatched to the 8 XCDs in turn (workgroup i to XCD
// i mod 8), and each XCD has its own L2.  With sm > 0 the tile grid is cut
// into sm row parts x (8 / sm) column parts and XCD x takes part x, its
// tiles in column-major order, so that each XCD's L2 holds only its part's
// operand rows and columns; the grid is 8 x the largest part, and a
// workgroup past its part's tile count has no tile.  sm = 0: row-major
// order over the whole grid (as a 2-D grid launch).  The mapping changes no
// tile's arithmetic.
__device__ __forceinline__ bool map_tile(int lin, int mt, int nt, int sm, int& tm, int& tn) {
    if (sm == 0) {
        tm = lin / nt;
        tn = lin - tm * nt;
        return tm < mt;
    }
    const int sn = 8 / sm, x = lin & 7, j = lin >> 3;
    const int xm = x / sn, xn = x - xm * sn;
    const int m_lo = xm * mt / sm, cm = (xm + 1) * mt / sm - m_lo;
    const int n_lo = xn * nt / sn, cn = (xn + 1) * nt / sn - n_lo;
    if (j >= cm * cn) return false;
    tm = m_lo + j % cm;
    tn = n_lo + j / cm;
    return true;
}

// Rows of A past M (the last row tile of a 128-row tiling) are read as row
// M - 1 and their outputs are not stored.
//
// KS > 1 splits each tile's K loop between KS groups of 4 waves in one
// workgroup (group g takes a contiguous share of the K stages, with its own
// LDS buffers and register ring); at the end the groups' accumulators are
// added in group order through LDS and group 0 applies the epilogue.  This
// doubles the waves in flight per tile for shapes whose tile count leaves
// CUs idle.  Every group runs the same number of loop trips (a group with
// fewer stages idles through its last ones), so the workgroup barriers match.
//
// PF is how many K stages ahead the global loads run (a ring of PF + 1
// register slots).  Two stages hide an L2 hit; operands that come from
// another XCD's L2 or from HBM need more.
template <int BM, int BN, int EPI, int KS = 1, int PF = 2>
__global__ __launch_bounds__(256 * KS) void k_gemm_nt(const uint16_t* __restrict__ A, int lda,
                                                      const uint16_t* __restrict__ B, int ldb, int M, int K,
                                                      const float* __restrict__ bias, void* __restrict__ Cout,
                                                      int ldc, const uint16_t* __restrict__ mask, int nt, int sm) {
    constexpr int BK = 64, LDK = BK + 8;
    constexpr int TM = BM / 64, TN = BN / 64;
    constexpr int CA = BM * BK / 8 / 256, CB = BN * BK / 8 / 256;
    __shared__ __align__(16) uint16_t sA[KS][2][BM * LDK];
    __shared__ __align__(16) uint16_t sB[KS][2][BN * LDK];
    const int grp = KS == 1 ? 0 : (int)(threadIdx.x >> 8);
    const int tid = KS == 1 ? (int)threadIdx.x : (int)(threadIdx.x & 255);
    const int lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;
    int tmi, tni;
    if (!map_tile((int)blockIdx.x, (M + BM - 1) / BM, nt, sm, tmi, tni)) return;
    const int64_t m0 = (int64_t)tmi * BM, n0 = (int64_t)tni * BN;
    // this group's K stages: [sbeg, sbeg + ng); every group loops `trips` times
    const int nk = K / BK;
    const int trips = KS == 1 ? nk : (nk + KS - 1) / KS;
    const int sbeg = KS == 1 ? 0 : grp * trips;
    const int ng = KS == 1 ? nk : max(0, min(nk - sbeg, trips));
    uint16_t(*gA)[BM * LDK] = sA[grp];
    uint16_t(*gB)[BN * LDK] = sB[grp];
    // Global -> register -> LDS pipeline.  Tiles are fetched two K-stages
    // ahead into a 3-slot register ring (slot indices are compile-time
    // constants after the 3-way unroll below, so the ring stays in
    // registers), stored to the idle LDS buffer one stage ahead, and consumed
    // from LDS by the MFMAs.
    constexpr int D = PF + 1;
    u32x4 ra[D][CA], rb[D][CB];
#define LN_GLOAD(slot, kt)                                                                         \
    do {                                                                                           \
        const int64_t k0 = (int64_t)(sbeg + (kt)) * BK;                                            \
        _Pragma("unroll") for (int i = 0; i < CA; i++) {                                           \
            const int c = tid + i * 256, row = c >> 3, col = (c & 7) * 8;                          \
            const int64_t ar = m0 + row < M ? m0 + row : M - 1;                                    \
            ra[slot][i] = *reinterpret_cast<const u32x4*>(A + ar * lda + k0 + col);                \
        }                                                                                          \
        _Pragma("unroll") for (int i = 0; i < CB; i++) {                                           \
            const int c = tid + i * 256, row = c >> 3, col = (c & 7) * 8;                          \
            rb[slot][i] = *reinterpret_cast<const u32x4*>(B + (n0 + row) * ldb + k0 + col);        \
        }                                                                                          \
    } while (0)
#define LN_SSTORE(slot, buf)                                                                       \
    do {                                                                                           \
        _Pragma("unroll") for (int i = 0; i < CA; i++) {                                           \
            const int c = tid + i * 256, row = c >> 3, col = (c & 7) * 8;                          \
            *reinterpret_cast<u32x4*>(&gA[buf][row * LDK + col]) = ra[slot][i];                    \
        }                                                                                          \
        _Pragma("unroll") for (int i = 0; i < CB; i++) {                                           \
            const int c = tid + i * 256, row = c >> 3, col = (c & 7) * 8;                          \
            *reinterpret_cast<u32x4*>(&gB[buf][row * LDK + col]) = rb[slot][i];                    \
        }                                                                                          \
    } while (0)
    // KACC independent accumulator chains per output tile, so consecutive
    // MFMAs of a wave do not wait on each other's results; summed at the end
    constexpr int KACC = (TM * TN >= 4) ? 1 : 4 / (TM * TN);
    v16f acc[KACC][TM][TN];
#pragma unroll
    for (int q = 0; q < KACC; q++)
#pragma unroll
        for (int i = 0; i < TM; i++)
#pragma unroll
            for (int j = 0; j < TN; j++)
#pragma unroll
                for (int r = 0; r < 16; r++) acc[q][i][j][r] = 0.f;
    const int kh = 8 * (lane >> 5), l32 = lane & 31;
    // Branch-free steady state (enough stages): every stage issues
    // its prefetch unconditionally, so the compiler can count the loads in
    // flight and wait for exactly the slot an LDS store needs; behind a
    // conditional prefetch it must assume the worst and wait for all of them.
    // (with KS groups, the steady loop runs the trip count of the group with
    // the fewest stages in every group, so that all take the same barriers)
    const int ng_min = KS == 1 ? nk : max(0, min(nk - (KS - 1) * trips, trips));
    const bool steady = ng_min >= PF + D;
    if (steady) {
#pragma unroll
        for (int q = 0; q < PF; q++) LN_GLOAD(q, q);
    } else {
        if (KS == 1 || ng > 0) LN_GLOAD(0, 0);
#pragma unroll
        for (int q = 1; q < PF; q++)
            if (ng > q) LN_GLOAD(q, q);
    }
    if (KS == 1 || ng > 0) LN_SSTORE(0, 0);
    __syncthreads();
#define LN_COMPUTE(buf)                                                                            \
    do {                                                                                           \
        v8bf fa[BK / 16][TM], fb[BK / 16][TN];                                                     \
        _Pragma("unroll") for (int kk = 0; kk < BK / 16; kk++) {                                   \
            _Pragma("unroll") for (int i = 0; i < TM; i++) fa[kk][i] = *reinterpret_cast<const v8bf*>( \
                &gA[buf][(wm * (BM / 2) + i * 32 + l32) * LDK + kk * 16 + kh]);                    \
            _Pragma("unroll") for (int j = 0; j < TN; j++) fb[kk][j] = *reinterpret_cast<const v8bf*>( \
                &gB[buf][(wn * (BN / 2) + j * 32 + l32) * LDK + kk * 16 + kh]);                    \
        }                                                                                          \
        _Pragma("unroll") for (int kk = 0; kk < BK / 16; kk++)                                     \
            _Pragma("unroll") for (int i = 0; i < TM; i++)                                         \
                _Pragma("unroll") for (int j = 0; j < TN; j++)                                     \
                    acc[kk % KACC][i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(               \
                        fa[kk][i], fb[kk][j], acc[kk % KACC][i][j], 0, 0, 0);                      \
    } while (0)
    // one stage: prefetch stage kt+PF into slot LSLOT, compute stage kt, move
    // stage kt+1 (slot SSLOT) into the other LDS buffer; stages past this
    // group's count are skipped but the barrier is still taken
    // The stage barrier orders LDS traffic only: this wave's LDS reads of the
    // buffer just consumed and its writes of the next one are complete
    // (lgkmcnt 0) before any wave passes.  __syncthreads() would also wait
    // for every global load in flight (vmcnt 0), i.e. for the prefetches
    // issued this very stage, and serialise the pipeline on memory latency;
    // the register-ring loads need no barrier, the compiler waits for each
    // slot before its LDS store.
#define LN_STAGE(kt, LSLOT, SSLOT)                                                                 \
    do {                                                                                           \
        if ((kt) + PF < ng) LN_GLOAD(LSLOT, (kt) + PF);                                            \
        if (KS == 1 || (kt) < ng) LN_COMPUTE((kt) & 1);                                            \
        if ((kt) + 1 < ng) LN_SSTORE(SSLOT, ((kt) + 1) & 1);                                       \
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");                            \
    } while (0)
#define LN_STAGE_STEADY(kt, LSLOT, SSLOT)                                                          \
    do {                                                                                           \
        LN_GLOAD(LSLOT, (kt) + PF);                                                                \
        LN_COMPUTE((kt) & 1);                                                                      \
        LN_SSTORE(SSLOT, ((kt) + 1) & 1);                                                          \
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");                            \
    } while (0)
    // unrolled D ways, so that every slot index is a compile-time constant
    int kt0 = 0;
    if (steady) {
        for (; kt0 + D <= ng_min - PF; kt0 += D) {
#pragma unroll
            for (int u = 0; u < D; u++) LN_STAGE_STEADY(kt0 + u, (u + PF) % D, (u + 1) % D);
        }
    }
    for (int kt = kt0; kt < trips; kt += D) {
#pragma unroll
        for (int u = 0; u < D; u++)
            if (kt + u < trips) LN_STAGE(kt + u, (u + PF) % D, (u + 1) % D);
    }
#undef LN_STAGE_STEADY
#undef LN_STAGE
#undef LN_COMPUTE
#undef LN_GLOAD
#undef LN_SSTORE
#pragma unroll
    for (int q = 1; q < KACC; q++)
#pragma unroll
        for (int i = 0; i < TM; i++)
#pragma unroll
            for (int j = 0; j < TN; j++)
#pragma unroll
                for (int r = 0; r < 16; r++) acc[0][i][j][r] += acc[q][i][j][r];
    if constexpr (KS > 1) {
        // groups 1.. hand their partial sums to group 0 through LDS, in group order
        float* xr = reinterpret_cast<float*>(&sA[0][0][0]);   // reused: all stages are done
        constexpr int PER = TM * TN * 16;                      // floats per lane
        for (int g = 1; g < KS; g++) {
            if (grp == g) {
#pragma unroll
                for (int i = 0; i < TM; i++)
#pragma unroll
                    for (int j = 0; j < TN; j++)
#pragma unroll
                        for (int r = 0; r < 16; r++) xr[((i * TN + j) * 16 + r) * 256 + tid] = acc[0][i][j][r];
            }
            __syncthreads();
            if (grp == 0) {
#pragma unroll
                for (int i = 0; i < TM; i++)
#pragma unroll
                    for (int j = 0; j < TN; j++)
#pragma unroll
                        for (int r = 0; r < 16; r++) acc[0][i][j][r] += xr[((i * TN + j) * 16 + r) * 256 + tid];
            }
            __syncthreads();
        }
        static_assert(PER * 256 * 4 <= (int)sizeof(sA), "partial sums must fit in the A buffers");
        if (grp != 0) return;
    }
#pragma unroll
    for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++) {
            const int64_t col = n0 + wn * (BN / 2) + j * 32 + l32;
            const float bv =
                (EPI == EPI_BIAS_F32 || EPI == EPI_BIAS_RELU_BF || EPI == EPI_BIAS_RELU_SWZ) ? bias[col] : 0.f;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int64_t row = m0 + wm * (BM / 2) + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row >= M) continue;
                float v = acc[0][i][j][r] + bv;
                if (EPI == EPI_BIAS_F32 || EPI == EPI_F32) {
                    reinterpret_cast<float*>(Cout)[row * ldc + col] = v;
                } else if (EPI == EPI_BIAS_RELU_BF) {
                    reinterpret_cast<uint16_t*>(Cout)[row * ldc + col] = f2bf(v > 0.f ? v : 0.f);
                } else if (EPI == EPI_BIAS_RELU_SWZ) {
                    reinterpret_cast<uint16_t*>(Cout)[swz_index(row, col, ldc)] = f2bf(v > 0.f ? v : 0.f);
                } else {
                    const bool on = bf2f(mask[row * ldc + col]) > 0.f;
                    reinterpret_cast<uint16_t*>(Cout)[row * ldc + col] = f2bf(on ? v : 0.f);
                }
            }
        }
}

// GEMM with both operands in the swizzled layout and no LDS stage: one wave
// per 64 x 64 output tile (2 x 2 MFMA tiles of 32 x 32), so every operand
// block feeds two MFMAs and a wave needs 1 KB of operands per MFMA, half of
// what a 32 x 32 wave tile needs.  Each operand block is one coalesced 1 KB
// load straight into registers, prefetched PF k-blocks ahead in a ring of
// PF + 1 slots; the loads are unconditional (clamped to the last block) so
// the compiler waits for exactly the slot it needs.  With KSPLIT = 2 or 4
// that many waves take equal shares of K and add their sums through LDS
// (wave 0 adds the others' in wave order).  K = 16 KBT is a compile-time
// constant; M and N are multiples of 64.
template <int EPI, int KSPLIT, int PF, int KBT>
__global__ __launch_bounds__(64 * KSPLIT) void k_gemm_direct(const uint16_t* __restrict__ A,
                                                            const uint16_t* __restrict__ B, int M,
                                                            const float* __restrict__ bias, void* __restrict__ Cout,
                                                            int ldc, int nt, int sm) {
    constexpr int D = PF + 1, KB = KBT, per = KBT / KSPLIT;
    static_assert(KBT % KSPLIT == 0 && per > PF, "k blocks per wave");
    const int lane = threadIdx.x & 63, grp = KSPLIT == 1 ? 0 : (int)(threadIdx.x >> 6);
    int tmi, tni;
    if (!map_tile((int)blockIdx.x, M / 64, nt, sm, tmi, tni)) return;
    const int64_t m0 = (int64_t)tmi * 64, n0 = (int64_t)tni * 64;
    const int64_t kb0 = (int64_t)grp * per;
    const v8bf* a0 = reinterpret_cast<const v8bf*>(A) + ((m0 >> 5) * KB + kb0) * 64 + lane;
    const v8bf* a1 = a0 + (int64_t)KB * 64;
    const v8bf* b0 = reinterpret_cast<const v8bf*>(B) + ((n0 >> 5) * KB + kb0) * 64 + lane;
    const v8bf* b1 = b0 + (int64_t)KB * 64;
    v8bf ra[D][2], rb[D][2];
    v16f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;
#define LD_BLOCKS(slot, kb)                                                                        \
    do {                                                                                           \
        const int64_t o = (int64_t)(kb) * 64;                                                      \
        ra[slot][0] = a0[o];                                                                       \
        ra[slot][1] = a1[o];                                                                       \
        rb[slot][0] = b0[o];                                                                       \
        rb[slot][1] = b1[o];                                                                       \
    } while (0)
#pragma unroll
    for (int q = 0; q < PF; q++) LD_BLOCKS(q, q);
    // fully unrolled (K is a compile-time constant): straight-line code, so
    // the compiler waits for exactly the ring slot each step consumes
#pragma unroll
    for (int kb = 0; kb < per; kb++) {
        if (kb + PF < per) LD_BLOCKS((kb + PF) % D, kb + PF);
        // keep the prefetch where it is: the scheduler would otherwise sink
        // the loads to their MFMAs and wait for each one
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int j = 0; j < 2; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ra[kb % D][i], rb[kb % D][j], acc[i][j], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
#undef LD_BLOCKS
    if constexpr (KSPLIT > 1) {
        // waves 1.. hand their partial sums to wave 0, which adds them in wave order
        __shared__ float xr[KSPLIT - 1][4 * 16 * 64];
        if (grp > 0) {
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
#pragma unroll
                    for (int r = 0; r < 16; r++) xr[grp - 1][((i * 2 + j) * 16 + r) * 64 + lane] = acc[i][j][r];
        }
        __syncthreads();
        if (grp != 0) return;
#pragma unroll
        for (int g = 0; g < KSPLIT - 1; g++)
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
#pragma unroll
                    for (int r = 0; r < 16; r++) acc[i][j][r] += xr[g][((i * 2 + j) * 16 + r) * 64 + lane];
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int64_t col = n0 + j * 32 + (lane & 31);
            const float bv = bias[col];
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int64_t row = m0 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row >= M) continue;
                const float v = acc[i][j][r] + bv;
                if (EPI == EPI_BIAS_F32) reinterpret_cast<float*>(Cout)[row * ldc + col] = v;
                else reinterpret_cast<uint16_t*>(Cout)[swz_index(row, col, ldc)] = f2bf(v > 0.f ? v : 0.f);
            }
        }
}

// Row-major bf16 [R][K] -> the swizzled layout, one 16-byte chunk per thread.
__global__ void k_swizzle_bf16(const uint16_t* __restrict__ in, int64_t R, int64_t K, uint16_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t q8 = K >> 3;
    if (i >= R * q8) return;
    const int64_t r = i / q8, k = (i - r * q8) * 8;
    *reinterpret_cast<u32x4*>(out + swz_index(r, k, K)) = *reinterpret_cast<const u32x4*>(in + r * K + k);
}

// bf16 transpose: out[c][r] = in[r][c], both dims multiples of 64.
__global__ __launch_bounds__(256) void k_transpose_bf16(const uint16_t* __restrict__ in, int ldin,
                                                        uint16_t* __restrict__ out, int ldout) {
    __shared__ uint16_t t[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) t[r][tx] = in[(r0 + r) * ldin + c0 + tx];
    __syncthreads();
    for (int c = ty; c < 64; c += 4) out[(c0 + c) * ldout + r0 + tx] = t[tx][c];
}

// fp32 -> bf16 copy of n elements
__global__ void k_to_bf16(const float* __restrict__ in, uint16_t* __restrict__ out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(in[i]);
}

// Rows [0, m) of a [rows][ld] fp32 matrix with `cols` valid columns -> bf16
// [rows][ldo]; rows >= m and columns >= cols become zero.
__global__ void k_rows_to_bf16(const float* __restrict__ in, int64_t m, int cols, uint16_t* __restrict__ out,
                               int ldo, int64_t rows) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * ldo) return;
    int64_t r = i / ldo;
    int c = (int)(i - r * ldo);
    out[i] = (r < m && c < cols) ? f2bf(in[r * cols + c]) : (uint16_t)0;
}

// Valid block of an fp32 [rows][ld] matrix -> dense [m][cols]
__global__ void k_unpad_f32(const float* __restrict__ in, int ld, int64_t m, int cols, float* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m * cols) return;
    int64_t r = i / cols;
    int c = (int)(i - r * cols);
    out[i] = in[r * ld + c];
}

// Sum of a mask -> 1 / max(sum, 1) in *inv (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void k_mask_inv(const float* __restrict__ mask, int64_t n, float* __restrict__ inv) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) s += mask[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) inv[0] = (float)(1.0 / (red[0] > 1.0 ? red[0] : 1.0));
}

// Huber loss (delta = 1) averaged over masked entries, its gradient as bf16
// [rows][ld] (zero outside the valid block), and per-block partial sums of
// the loss for a deterministic final reduction.
__global__ __launch_bounds__(256) void k_huber(const float* __restrict__ y, int ld, const float* __restrict__ t,
                                               const float* __restrict__ mask, int64_t m, int cols,
                                               const float* __restrict__ inv_n_p, uint16_t* __restrict__ g,
                                               int64_t rows, double* __restrict__ part) {
    __shared__ double red[256];
    const float inv_n = inv_n_p[0];
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double l = 0.0;
    if (i < rows * ld) {
        int64_t r = i / ld;
        int c = (int)(i - r * ld);
        float gv = 0.f;
        if (r < m && c < cols) {
            int64_t k = r * cols + c;
            float mk = mask[k];
            float d = (y[i] - t[k]) * mk;
            float a = fabsf(d);
            l = a <= 1.f ? 0.5 * (double)d * d : (double)a - 0.5;
            gv = (a <= 1.f ? d : copysignf(1.f, d)) * inv_n;
        }
        g[i] = f2bf(gv);
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Column sums of a bf16 [rows][ld] matrix -> fp32 [ld] (bias gradients).
__global__ __launch_bounds__(256) void k_colsum_bf16(const uint16_t* __restrict__ g, int ld, int64_t rows,
                                                     float* __restrict__ out) {
    int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= ld) return;
    float s = 0.f;
    for (int64_t r = 0; r < rows; r++) s += bf2f(g[r * ld + c]);
    out[c] = s;
}

// Adam (Kingma & Ba) on FP32 masters, refreshing the bf16 copy; `live`
// marks entries that are real parameters (padding stays zero).
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ pb, const uint8_t* __restrict__ live, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !live[i]) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    pb[i] = f2bf(pi);
}

// ------------------------------------------------------------------ host
static int32_t hipchk(hipError_t e, const char* what) {
    if (e == hipSuccess) return PCFR_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return PCFR_E_DEVICE;
}
#define LN_CHK(call)                                        \
    do {                                                    \
        int32_t _rc = hipchk((call), #call);                \
        if (_rc != PCFR_OK) return _rc;                     \
    } while (0)

static int64_t r64(int64_t x) { return (x + 63) / 64 * 64; }

// XCD split of an mt x nt tile grid for map_tile: the row-part count sm
// (1, 2, 4 or 8; 0 = no split for grids too small to share) that minimises
// the operand rows plus columns one XCD touches, and the grid it needs.
static void tile_grid(int64_t mt, int64_t nt, int64_t BM, int64_t BN, int* sm, int64_t* grid) {
    *sm = 0;
    *grid = mt * nt;
    if (mt * nt < 32) return;
    int64_t best = -1;
    for (int s = 1; s <= 8; s *= 2) {
        const int sn = 8 / s;
        if (mt < s || nt < sn) continue;
        const int64_t cm = (mt + s - 1) / s, cn = (nt + sn - 1) / sn;
        const int64_t foot = cm * BM + cn * BN;
        if (best < 0 || foot < best) { best = foot; *sm = s; *grid = 8 * cm * cn; }
    }
}
static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

bool gemm_tile_valid(int tile, int64_t N) {
    static const int bn[kGemmTiles] = {64, 64, 128, 128, 64, 128, 64, 128, 64, 64, 64};
    return tile >= 0 && tile < kGemmTiles && N % bn[tile] == 0;
}

constexpr int kDirectPF = 7;    // prefetch distance of the DIRECT tiles, in k-blocks of 16
constexpr int kDirectKB = 96;   // their input width in k-blocks (1536, the hidden width)

bool gemm_tile_valid_layer(int tile, int l, int64_t N, int64_t K) {
    if (!gemm_tile_valid(tile, N)) return false;
    if (!gemm_tile_direct(tile)) return true;
    return l > 0 && K == 16 * kDirectKB;
}

// C = A B^T with both operands swizzled (M, N multiples of 64); out_swz: the
// bf16 ReLU output swizzled for the next layer, else the FP32 output row-major.
static int32_t launch_gemm_direct(hipStream_t st, int tile, const uint16_t* A, const uint16_t* B, int64_t M,
                                  int64_t N, int64_t K, const float* bias, void* C, int ldc, bool relu_swz) {
    if (K != 16 * kDirectKB) { set_error("direct tiles need an input width of 1536"); return PCFR_E_INVALID_ARG; }
    int sm;
    int64_t ng;
    tile_grid(M / 64, N / 64, 64, 64, &sm, &ng);
    const dim3 grid((unsigned)ng);
    const int nt = (int)(N / 64);
    const int ks = tile == GEMM_DIRECT_K4 ? 4 : tile == GEMM_DIRECT_K2 ? 2 : 1;
#define LN_DIRECT(E, KSv)                                                                                  \
    hipLaunchKernelGGL((k_gemm_direct<E, KSv, kDirectPF, kDirectKB>), grid, dim3(64 * KSv), 0, st, A, B, (int)M, \
                       bias, C, ldc, nt, sm)
    if (relu_swz) {
        if (ks == 1) LN_DIRECT(EPI_BIAS_RELU_SWZ, 1);
        else if (ks == 2) LN_DIRECT(EPI_BIAS_RELU_SWZ, 2);
        else LN_DIRECT(EPI_BIAS_RELU_SWZ, 4);
    } else {
        if (ks == 1) LN_DIRECT(EPI_BIAS_F32, 1);
        else if (ks == 2) LN_DIRECT(EPI_BIAS_F32, 2);
        else LN_DIRECT(EPI_BIAS_F32, 4);
    }
#undef LN_DIRECT
    return hipchk(hipGetLastError(), "direct gemm launch");
}

int32_t launch_gemm(hipStream_t st, int epi, const uint16_t* A, int lda, const uint16_t* B, int ldb, int64_t M,
                    int64_t N, int64_t K, const float* bias, void* C, int ldc, const uint16_t* mask, int tile) {
    if (M % 64 || N % 64 || K % 64 || M <= 0 || N <= 0 || K <= 0) {
        set_error("GEMM dims must be positive multiples of 64");
        return PCFR_E_INVALID_ARG;
    }
    if (tile < 0) {
        // default: 128 x 128 tiles when they still give at least one workgroup per CU
        tile = (M % 128 == 0) && (N % 128 == 0) && (M / 128) * (N / 128) >= 256 ? GEMM_128x128 : GEMM_64x64;
    }
    if (!gemm_tile_valid(tile, N)) { set_error("GEMM tile does not divide N"); return PCFR_E_INVALID_ARG; }
#define LN_GEMM(BMv, BNv, E, KSv, PFv)                                                                   \
    do {                                                                                                 \
        int sm_;                                                                                         \
        int64_t ng_;                                                                                     \
        tile_grid((M + BMv - 1) / BMv, N / BNv, BMv, BNv, &sm_, &ng_);                                    \
        hipLaunchKernelGGL((k_gemm_nt<BMv, BNv, E, KSv, PFv>), dim3((unsigned)ng_), dim3(256 * KSv), 0, st, \
                           A, lda, B, ldb, (int)M, (int)K, bias, C, ldc, mask, (int)(N / BNv), sm_);      \
    } while (0)
#define LN_EPI(BMv, BNv, KSv, PFv)                                                       \
    switch (epi) {                                                                       \
        case EPI_BIAS_F32: LN_GEMM(BMv, BNv, EPI_BIAS_F32, KSv, PFv); break;             \
        case EPI_BIAS_RELU_BF: LN_GEMM(BMv, BNv, EPI_BIAS_RELU_BF, KSv, PFv); break;     \
        case EPI_F32: LN_GEMM(BMv, BNv, EPI_F32, KSv, PFv); break;                       \
        case EPI_BIAS_RELU_SWZ: LN_GEMM(BMv, BNv, EPI_BIAS_RELU_SWZ, KSv, PFv); break;   \
        default: LN_GEMM(BMv, BNv, EPI_MASK_BF, KSv, PFv); break;                        \
    }
    switch (tile) {
        case GEMM_64x64: LN_EPI(64, 64, 1, 2); break;
        case GEMM_128x64: LN_EPI(128, 64, 1, 2); break;
        case GEMM_64x128: LN_EPI(64, 128, 1, 2); break;
        case GEMM_128x128: LN_EPI(128, 128, 1, 2); break;
        case GEMM_64x64_K2: LN_EPI(64, 64, 2, 2); break;
        case GEMM_64x128_K2: LN_EPI(64, 128, 2, 2); break;
        case GEMM_64x64_P4: LN_EPI(64, 64, 1, 4); break;
        case GEMM_64x128_P4: LN_EPI(64, 128, 1, 4); break;
        default: set_error("direct tiles are launched through launch_gemm_direct"); return PCFR_E_INVALID_ARG;
    }
#undef LN_EPI
#undef LN_GEMM
    return hipchk(hipGetLastError(), "gemm launch");
}

static int32_t transpose(hipStream_t st, const uint16_t* in, int64_t rows, int64_t cols, uint16_t* out) {
    hipLaunchKernelGGL(k_transpose_bf16, dim3((unsigned)(cols / 64), (unsigned)(rows / 64)), dim3(256), 0, st, in,
                       (int)cols, out, (int)rows);
    return hipchk(hipGetLastError(), "transpose launch");
}

void LeafNetPlan::make(int d_in_, int width_, int depth_, int d_out_, int max_batch_) {
    d_in = d_in_; width = width_; depth = depth_; d_out = d_out_;
    Mp = r64(max_batch_);
    L = depth + 1;
    dims.assign(L + 1, 0);
    pdims.assign(L + 1, 0);
    dims[0] = d_in;
    for (int i = 1; i < L; i++) dims[i] = width;
    dims[L] = d_out;
    for (int i = 0; i <= L; i++) pdims[i] = r64(dims[i]);
    woff.assign(L, 0);
    boff.assign(L, 0);
    int64_t o = 0;
    for (int l = 0; l < L; l++) {
        woff[l] = o;
        o += pdims[l + 1] * pdims[l];
        boff[l] = o;
        o += pdims[l + 1];
    }
    n_padded = o;
    n_params = 0;
    for (int l = 0; l < L; l++) n_params += (int64_t)dims[l + 1] * dims[l] + dims[l + 1];
    maxw = 0;
    for (int i = 0; i <= L; i++) maxw = std::max<int64_t>(maxw, pdims[i]);
    size_t s = 0;
    auto take = [&](size_t b) { size_t at = s; s = a256(s + b); return at; };
    off_p = take(4 * n_padded);
    off_pb = take(2 * n_padded);
    off_pbs = take(2 * n_padded);
    off_g = take(4 * n_padded);
    off_m = take(4 * n_padded);
    off_v = take(4 * n_padded);
    off_live = take(n_padded);
    off_wt = take(2 * (size_t)maxw * maxw);
    off_x = take(2 * (size_t)Mp * pdims[0]);
    off_h.assign(L, 0);
    for (int l = 1; l < L; l++) off_h[l] = take(2 * (size_t)Mp * pdims[l]);
    off_y = take(4 * (size_t)Mp * pdims[L]);
    off_dz = take(2 * (size_t)Mp * maxw);
    off_dz2 = take(2 * (size_t)Mp * maxw);
    off_t1 = take(2 * (size_t)Mp * maxw);
    off_t2 = take(2 * (size_t)Mp * maxw);
    off_part = take(8 * (size_t)((Mp * pdims[L] + 255) / 256));
    off_cnt = take(16);
    total = s;
}

static int32_t swizzle_weights(pcfr_leafnet* n, hipStream_t st);   // below, with the forward

}  // namespace pcfr

using namespace pcfr;

extern "C" {

int32_t pcfr_leafnet_workspace_bytes(int32_t d_in, int32_t width, int32_t depth, int32_t d_out, int32_t max_batch,
                                     size_t* bytes) {
    if (!bytes || d_in <= 0 || width <= 0 || depth < 1 || depth > 16 || d_out <= 0 || max_batch <= 0) {
        set_error("invalid network shape");
        return PCFR_E_INVALID_ARG;
    }
    LeafNetPlan p;
    p.make(d_in, width, depth, d_out, max_batch);
    *bytes = p.total;
    return PCFR_OK;
}

int32_t pcfr_leafnet_create(int32_t d_in, int32_t width, int32_t depth, int32_t d_out, int32_t max_batch,
                            void* workspace, size_t bytes, void* stream, pcfr_leafnet** out) {
    size_t need;
    int32_t rc = pcfr_leafnet_workspace_bytes(d_in, width, depth, d_out, max_batch, &need);
    if (rc) return rc;
    if (!workspace || !out) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) { set_error("workspace must be 256-byte aligned"); return PCFR_E_INVALID_ARG; }
    if (bytes < need) { set_error("workspace smaller than pcfr_leafnet_workspace_bytes"); return PCFR_E_OUT_OF_MEMORY; }
    pcfr_leafnet* n = new (std::nothrow) pcfr_leafnet;
    if (!n) { set_error("out of host memory"); return PCFR_E_OUT_OF_MEMORY; }
    n->P.make(d_in, width, depth, d_out, max_batch);
    n->ws = reinterpret_cast<char*>(workspace);
    n->stream = reinterpret_cast<hipStream_t>(stream);
    const LeafNetPlan& P = n->P;
    rc = hipchk(hipMemsetAsync(n->ws, 0, P.total, n->stream), "workspace clear");
    if (rc) { delete n; return rc; }
    std::vector<uint8_t> live(P.n_padded, 0);
    for (int l = 0; l < P.L; l++) {
        for (int o = 0; o < P.dims[l + 1]; o++) {
            for (int i = 0; i < P.dims[l]; i++) live[P.woff[l] + (int64_t)o * P.pdims[l] + i] = 1;
            live[P.boff[l] + o] = 1;
        }
    }
    rc = hipchk(hipMemcpyAsync(n->ws + P.off_live, live.data(), live.size(), hipMemcpyHostToDevice, n->stream), "upload");
    if (!rc) rc = hipchk(hipStreamSynchronize(n->stream), "sync");
    if (rc) { delete n; return rc; }
    *out = n;
    return PCFR_OK;
}

int32_t pcfr_leafnet_free(pcfr_leafnet* n) {
    if (!n) return PCFR_OK;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    delete n;
    return PCFR_OK;
}

int32_t pcfr_leafnet_num_params(const pcfr_leafnet* n, int64_t* count) {
    if (!n || !count) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    *count = n->P.n_params;
    return PCFR_OK;
}

// Host parameter layout: for each layer l, W_l [out][in] row-major, then b_l [out].
int32_t pcfr_leafnet_set_params(pcfr_leafnet* n, const float* host) {
    if (!n || !host) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    const LeafNetPlan& P = n->P;
    std::vector<float> pad(P.n_padded, 0.f);
    int64_t k = 0;
    for (int l = 0; l < P.L; l++) {
        for (int o = 0; o < P.dims[l + 1]; o++)
            for (int i = 0; i < P.dims[l]; i++) {
                float v = host[k++];
                if (!std::isfinite(v)) { set_error("non-finite parameter"); return PCFR_E_INVALID_ARG; }
                pad[P.woff[l] + (int64_t)o * P.pdims[l] + i] = v;
            }
        for (int o = 0; o < P.dims[l + 1]; o++) {
            float v = host[k++];
            if (!std::isfinite(v)) { set_error("non-finite parameter"); return PCFR_E_INVALID_ARG; }
            pad[P.boff[l] + o] = v;
        }
    }
    LN_CHK(hipMemcpyAsync(n->ws + P.off_p, pad.data(), 4 * P.n_padded, hipMemcpyHostToDevice, n->stream));
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((P.n_padded + 255) / 256)), dim3(256), 0, n->stream,
                       reinterpret_cast<float*>(n->ws + P.off_p), reinterpret_cast<uint16_t*>(n->ws + P.off_pb),
                       P.n_padded);
    LN_CHK(hipGetLastError());
    if (int32_t rc = swizzle_weights(n, n->stream)) return rc;
    LN_CHK(hipMemsetAsync(n->ws + P.off_m, 0, 4 * P.n_padded, n->stream));
    LN_CHK(hipMemsetAsync(n->ws + P.off_v, 0, 4 * P.n_padded, n->stream));
    n->adam_t = 0;
    LN_CHK(hipStreamSynchronize(n->stream));
    return PCFR_OK;
}

static int32_t get_padded(pcfr_leafnet* n, size_t off, float* host) {
    const LeafNetPlan& P = n->P;
    std::vector<float> pad(P.n_padded);
    LN_CHK(hipMemcpyAsync(pad.data(), n->ws + off, 4 * P.n_padded, hipMemcpyDeviceToHost, n->stream));
    LN_CHK(hipStreamSynchronize(n->stream));
    int64_t k = 0;
    for (int l = 0; l < P.L; l++) {
        for (int o = 0; o < P.dims[l + 1]; o++)
            for (int i = 0; i < P.dims[l]; i++) host[k++] = pad[P.woff[l] + (int64_t)o * P.pdims[l] + i];
        for (int o = 0; o < P.dims[l + 1]; o++) host[k++] = pad[P.boff[l] + o];
    }
    return PCFR_OK;
}

int32_t pcfr_leafnet_get_params(pcfr_leafnet* n, float* host) {
    if (!n || !host) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    return get_padded(n, n->P.off_p, host);
}

int32_t pcfr_leafnet_get_grads(pcfr_leafnet* n, float* host) {
    if (!n || !host) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    return get_padded(n, n->P.off_g, host);
}

}  // extern "C"

namespace pcfr {

// Forward over the rows already staged in the bf16 input buffer; M = padded rows.
// Forward layer l on the first M rows of the staged activations.
// The tile layer l runs with: its chosen tile, or the default where direct
// tiles are not allowed.
static int layer_tile(const pcfr_leafnet* n, int l, bool allow_direct) {
    const int t = l < (int)n->fwd_tile.size() ? n->fwd_tile[l] : -1;
    return (gemm_tile_direct(t) && !allow_direct) ? -1 : t;
}

// Layer l with `tile`; its input is swizzled when the tile is direct, its
// hidden output swizzled when the next layer's tile (next_tile) is direct.
static int32_t forward_layer(pcfr_leafnet* n, int l, int64_t M, hipStream_t st, int tile, int next_tile) {
    const LeafNetPlan& P = n->P;
    const uint16_t* in = reinterpret_cast<const uint16_t*>(n->ws + (l == 0 ? P.off_x : P.off_h[l]));
    const float* b = reinterpret_cast<const float*>(n->ws + P.off_p) + P.boff[l];
    const bool hidden = l + 1 < P.L;
    void* out = hidden ? (void*)(n->ws + P.off_h[l + 1]) : (void*)(n->ws + P.off_y);
    if (gemm_tile_direct(tile)) {
        if (!gemm_tile_valid_layer(tile, l, P.pdims[l + 1], P.pdims[l]) || M % 64) {
            set_error("direct tile not valid for this layer");
            return PCFR_E_INVALID_ARG;
        }
        const uint16_t* Ws = reinterpret_cast<const uint16_t*>(n->ws + P.off_pbs) + P.woff[l];
        if (hidden && !gemm_tile_direct(next_tile)) {
            set_error("a direct layer's output feeds a direct layer only");
            return PCFR_E_INVALID_ARG;
        }
        return launch_gemm_direct(st, tile, in, Ws, M, P.pdims[l + 1], P.pdims[l], b, out, (int)P.pdims[l + 1], hidden);
    }
    const uint16_t* W = reinterpret_cast<const uint16_t*>(n->ws + P.off_pb) + P.woff[l];
    const int epi = !hidden ? EPI_BIAS_F32 : gemm_tile_direct(next_tile) ? EPI_BIAS_RELU_SWZ : EPI_BIAS_RELU_BF;
    return launch_gemm(st, epi, in, (int)P.pdims[l], W, (int)P.pdims[l], M, P.pdims[l + 1], P.pdims[l], b, out,
                       (int)P.pdims[l + 1], nullptr, tile);
}

int32_t leafnet_forward_staged(pcfr_leafnet* n, int64_t M, hipStream_t st, LaunchTimer* tm, bool allow_direct) {
    const LeafNetPlan& P = n->P;
    for (int l = 0; l < P.L; l++) {
        if (tm) tm->before(l + 1 < P.L ? 5 : 6);
        const int32_t rc = forward_layer(n, l, M, st, layer_tile(n, l, allow_direct),
                                         l + 1 < P.L ? layer_tile(n, l + 1, allow_direct) : -1);
        if (tm) tm->after();
        if (rc) return rc;
    }
    return PCFR_OK;
}

// Swizzled copies of the bf16 weights, for the direct tiles.
static int32_t swizzle_weights(pcfr_leafnet* n, hipStream_t st) {
    const LeafNetPlan& P = n->P;
    for (int l = 0; l < P.L; l++) {
        const int64_t R = P.pdims[l + 1], K = P.pdims[l], chunks = R * K / 8;
        hipLaunchKernelGGL(k_swizzle_bf16, dim3((unsigned)((chunks + 255) / 256)), dim3(256), 0, st,
                           reinterpret_cast<const uint16_t*>(n->ws + P.off_pb) + P.woff[l], R, K,
                           reinterpret_cast<uint16_t*>(n->ws + P.off_pbs) + P.woff[l]);
    }
    return hipchk(hipGetLastError(), "weight swizzle");
}

// Average ms of `reps` back-to-back runs of fn() on the net's stream.
template <typename F>
static int32_t time_ms(hipStream_t st, int reps, double* ms, F fn) {
    hipEvent_t a = nullptr, b = nullptr;
    LN_CHK(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) { (void)hipEventDestroy(a); return hipchk(e, "hipEventCreate"); }
    int32_t rc = fn();                      // untimed first run
    if (rc == PCFR_OK) e = hipEventRecord(a, st);
    for (int r = 0; r < reps && rc == PCFR_OK && e == hipSuccess; r++) rc = fn();
    if (rc == PCFR_OK && e == hipSuccess) e = hipEventRecord(b, st);
    if (rc == PCFR_OK && e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0;
    if (rc == PCFR_OK && e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    LN_CHK(e);
    *ms = (double)t / std::max(reps, 1);
    return PCFR_OK;
}

// Tile autotuner of the forward GEMMs for M rows: each layer is timed with
// every tile that divides its output width and keeps the fastest.  Tiles
// differ in how many partial-sum chains an output's K range is split into, so
// outputs may change in the last bits with the choice (fixed once made).
int32_t leafnet_autotune(pcfr_leafnet* n, int64_t M, int reps, double* ms_before, double* ms_after) {
    const LeafNetPlan& P = n->P;
    if (M <= 0 || M > P.Mp || M % 64) { set_error("autotune rows must be a multiple of 64 within max_batch"); return PCFR_E_INVALID_ARG; }
    hipStream_t st = n->stream;
    int32_t rc = time_ms(st, reps, ms_before, [&] { return leafnet_forward_staged(n, M, st); });
    if (rc) return rc;
    // Layers are timed one at a time (their inputs' contents do not matter
    // for timing).  Direct tiles need the layers after them direct too (a
    // direct layer writes swizzled output), so they are chosen as a suffix:
    // the best first layer of the suffix is decided by comparing, for every
    // split, the LDS-staged prefix plus the direct suffix.
    std::vector<int> pick(P.L, -1);
    std::vector<double> best_std(P.L, 1e30), best_dir(P.L, 1e30);
    std::vector<int> tile_std(P.L, -1), tile_dir(P.L, -1);
    for (int l = 0; l < P.L; l++) {
        for (int tile = 0; tile < kGemmTiles; tile++) {
            if (!gemm_tile_valid_layer(tile, l, P.pdims[l + 1], P.pdims[l])) continue;
            const bool dir = gemm_tile_direct(tile);
            double ms = 0;
            if ((rc = time_ms(st, reps, &ms, [&] { return forward_layer(n, l, M, st, tile, dir ? tile : -1); })))
                return rc;
            if (dir && ms < best_dir[l]) { best_dir[l] = ms; tile_dir[l] = tile; }
            if (!dir && ms < best_std[l]) { best_std[l] = ms; tile_std[l] = tile; }
        }
    }
    int split = P.L;   // layers [split, L) run direct
    double best_total = 1e30;
    for (int sp = 1; sp <= P.L; sp++) {
        double t = 0;
        bool ok = true;
        for (int l = 0; l < P.L; l++) {
            const double v = l < sp ? best_std[l] : best_dir[l];
            if (!(v < 1e29)) { ok = false; break; }
            t += v;
        }
        if (ok && t < best_total) { best_total = t; split = sp; }
    }
    for (int l = 0; l < P.L; l++) pick[l] = l < split ? tile_std[l] : tile_dir[l];
    n->fwd_tile = pick;
    return time_ms(st, reps, ms_after, [&] { return leafnet_forward_staged(n, M, st); });
}

}  // namespace pcfr

extern "C" {

int32_t pcfr_leafnet_set_tiles(pcfr_leafnet* n, const int32_t* tiles, int32_t count) {
    if (!n || !tiles) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    const LeafNetPlan& P = n->P;
    if (count != P.L) { set_error("one tile per layer is needed"); return PCFR_E_INVALID_ARG; }
    for (int l = 0; l < P.L; l++) {
        if (tiles[l] != -1 && !gemm_tile_valid_layer(tiles[l], l, P.pdims[l + 1], P.pdims[l])) {
            set_error("tile does not divide the layer's output width, or a direct tile on the first layer");
            return PCFR_E_INVALID_ARG;
        }
        if (l + 1 < P.L && gemm_tile_direct(tiles[l]) && !gemm_tile_direct(tiles[l + 1])) {
            set_error("a direct tile must be followed by direct tiles");
            return PCFR_E_INVALID_ARG;
        }
    }
    n->fwd_tile.assign(tiles, tiles + count);
    return PCFR_OK;
}

int32_t pcfr_leafnet_get_tiles(pcfr_leafnet* n, int32_t* tiles, int32_t count) {
    if (!n || !tiles) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    if (count != n->P.L) { set_error("one tile per layer is needed"); return PCFR_E_INVALID_ARG; }
    for (int l = 0; l < count; l++) tiles[l] = l < (int)n->fwd_tile.size() ? n->fwd_tile[l] : -1;
    return PCFR_OK;
}

int32_t pcfr_leafnet_autotune(pcfr_leafnet* n, int32_t m, int32_t reps, double* ms_before, double* ms_after) {
    if (!n || m <= 0 || reps < 1 || !ms_before || !ms_after) { set_error("null argument, empty batch or reps < 1"); return PCFR_E_INVALID_ARG; }
    if (m > n->P.Mp) { set_error("batch larger than max_batch"); return PCFR_E_INVALID_ARG; }
    return leafnet_autotune(n, r64(m), reps, ms_before, ms_after);
}

int32_t pcfr_leafnet_forward(pcfr_leafnet* n, const float* x, int32_t m, float* y) {
    if (!n || !x || !y || m <= 0) { set_error("null argument or empty batch"); return PCFR_E_INVALID_ARG; }
    const LeafNetPlan& P = n->P;
    if (m > P.Mp) { set_error("batch larger than max_batch"); return PCFR_E_INVALID_ARG; }
    const int64_t M = r64(m);
    const int64_t tot = M * P.pdims[0];
    hipLaunchKernelGGL(k_rows_to_bf16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, n->stream, x, (int64_t)m,
                       P.dims[0], reinterpret_cast<uint16_t*>(n->ws + P.off_x), (int)P.pdims[0], M);
    LN_CHK(hipGetLastError());
    int32_t rc = leafnet_forward_staged(n, M, n->stream);
    if (rc) return rc;
    const int64_t ny = (int64_t)m * P.dims[P.L];
    hipLaunchKernelGGL(k_unpad_f32, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, n->stream,
                       reinterpret_cast<const float*>(n->ws + P.off_y), (int)P.pdims[P.L], (int64_t)m, P.dims[P.L], y);
    LN_CHK(hipGetLastError());
    return PCFR_OK;
}

// One Adam step on the Huber loss of a batch: forward, loss gradient,
// backward GEMMs (dW = dZ^T H, dH = dZ W masked by the ReLU), bias sums,
// Adam.  x [m][d_in], target and mask [m][d_out] are device fp32.
int32_t pcfr_leafnet_train_step(pcfr_leafnet* n, const float* x, const float* target, const float* mask, int32_t m,
                                float lr, float* loss) {
    if (!n || !x || !target || !mask || m <= 0) { set_error("null argument or empty batch"); return PCFR_E_INVALID_ARG; }
    const LeafNetPlan& P = n->P;
    if (m > P.Mp) { set_error("batch larger than max_batch"); return PCFR_E_INVALID_ARG; }
    hipStream_t st = n->stream;
    const int64_t M = r64(m);
    {
        const int64_t tot = M * P.pdims[0];
        hipLaunchKernelGGL(k_rows_to_bf16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, x, (int64_t)m,
                           P.dims[0], reinterpret_cast<uint16_t*>(n->ws + P.off_x), (int)P.pdims[0], M);
        LN_CHK(hipGetLastError());
    }
    int32_t rc = leafnet_forward_staged(n, M, st, nullptr, false);
    if (rc) return rc;
    const int64_t ny = (int64_t)m * P.dims[P.L];
    float* inv_n = reinterpret_cast<float*>(n->ws + P.off_cnt);
    hipLaunchKernelGGL(k_mask_inv, dim3(1), dim3(1024), 0, st, mask, ny, inv_n);
    LN_CHK(hipGetLastError());
    const int64_t Ny = P.pdims[P.L];
    const int64_t nel = M * Ny;
    const unsigned nblk = (unsigned)((nel + 255) / 256);
    uint16_t* dz = reinterpret_cast<uint16_t*>(n->ws + P.off_dz);
    uint16_t* dz2 = reinterpret_cast<uint16_t*>(n->ws + P.off_dz2);
    uint16_t* t1 = reinterpret_cast<uint16_t*>(n->ws + P.off_t1);
    uint16_t* t2 = reinterpret_cast<uint16_t*>(n->ws + P.off_t2);
    uint16_t* wt = reinterpret_cast<uint16_t*>(n->ws + P.off_wt);
    float* g = reinterpret_cast<float*>(n->ws + P.off_g);
    double* part = reinterpret_cast<double*>(n->ws + P.off_part);
    hipLaunchKernelGGL(k_huber, dim3(nblk), dim3(256), 0, st, reinterpret_cast<const float*>(n->ws + P.off_y),
                       (int)Ny, target, mask, (int64_t)m, P.dims[P.L], inv_n, dz, M, part);
    LN_CHK(hipGetLastError());
    for (int l = P.L - 1; l >= 0; l--) {
        const int64_t in = P.pdims[l], outd = P.pdims[l + 1];
        const uint16_t* H = l == 0 ? reinterpret_cast<const uint16_t*>(n->ws + P.off_x)
                                   : reinterpret_cast<const uint16_t*>(n->ws + P.off_h[l]);
        // dW_l = dZ^T H: A' = dZ^T [out][M], B' = H^T [in][M]
        if ((rc = transpose(st, dz, M, outd, t1))) return rc;
        if ((rc = transpose(st, H, M, in, t2))) return rc;
        if ((rc = launch_gemm(st, EPI_F32, t1, (int)M, t2, (int)M, outd, in, M, nullptr, g + P.woff[l], (int)in,
                              nullptr)))
            return rc;
        hipLaunchKernelGGL(k_colsum_bf16, dim3((unsigned)((outd + 255) / 256)), dim3(256), 0, st, dz, (int)outd, M,
                           g + P.boff[l]);
        LN_CHK(hipGetLastError());
        if (l > 0) {
            // dZ_{l-1} = (dZ_l W_l) * [H_l > 0]: B' = W_l^T [in][out]
            const uint16_t* W = reinterpret_cast<const uint16_t*>(n->ws + P.off_pb) + P.woff[l];
            if ((rc = transpose(st, W, outd, in, wt))) return rc;
            if ((rc = launch_gemm(st, EPI_MASK_BF, dz, (int)outd, wt, (int)outd, M, in, outd, nullptr, dz2, (int)in,
                                  H)))
                return rc;
            std::swap(dz, dz2);
        }
    }
    n->adam_t++;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)n->adam_t), c2 = 1.f - powf(b2, (float)n->adam_t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((P.n_padded + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<float*>(n->ws + P.off_p), g, reinterpret_cast<float*>(n->ws + P.off_m),
                       reinterpret_cast<float*>(n->ws + P.off_v), reinterpret_cast<uint16_t*>(n->ws + P.off_pb),
                       reinterpret_cast<const uint8_t*>(n->ws + P.off_live), P.n_padded, lr, b1, b2, eps, c1, c2);
    LN_CHK(hipGetLastError());
    if ((rc = swizzle_weights(n, st))) return rc;
    if (loss) {
        std::vector<double> hp(nblk);
        float iv = 1.f;
        LN_CHK(hipMemcpyAsync(hp.data(), part, 8 * nblk, hipMemcpyDeviceToHost, st));
        LN_CHK(hipMemcpyAsync(&iv, inv_n, 4, hipMemcpyDeviceToHost, st));
        LN_CHK(hipStreamSynchronize(st));
        double s = 0;
        for (double v : hp) s += v;
        *loss = (float)(s * iv);
    }
    return PCFR_OK;
}

}  // extern "C"
