// Leaf network: workspace plan and handle (shared by the solver's leaf stage).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "../../include/pcfr.h"

namespace pcfr {

struct LeafNetPlan {
    int d_in = 0, width = 0, depth = 0, d_out = 0, L = 0;
    int64_t Mp = 0;                       // max batch rows, padded to 64
    std::vector<int> dims;                // layer widths, unpadded (L + 1)
    std::vector<int64_t> pdims;           // padded to 64
    std::vector<int64_t> woff, boff;      // parameter offsets (elements) in the padded layout
    int64_t n_padded = 0, n_params = 0, maxw = 0;
    size_t off_p = 0, off_pb = 0, off_pbs = 0, off_g = 0, off_m = 0, off_v = 0, off_live = 0, off_wt = 0, off_x = 0;
    std::vector<size_t> off_h;            // hidden activations (bf16), index 1..L-1
    size_t off_y = 0, off_dz = 0, off_dz2 = 0, off_t1 = 0, off_t2 = 0, off_part = 0, off_cnt = 0, total = 0;
    void make(int d_in, int width, int depth, int d_out, int max_batch);
};

// GEMM workgroup tiles (rows x columns of C); 4 waves, each a quarter tile;
// the _K2 variants run two such groups that split K (8 waves).  The DIRECT
// tiles read both operands in the swizzled layout with no LDS stage, one
// wave (two with _K2, four with _K4, splitting K) per 64 x 64 tile; a layer
// using them needs its input written swizzled by the layer before, so never
// the first layer.
enum {
    GEMM_64x64 = 0, GEMM_128x64 = 1, GEMM_64x128 = 2, GEMM_128x128 = 3, GEMM_64x64_K2 = 4, GEMM_64x128_K2 = 5,
    GEMM_64x64_P4 = 6, GEMM_64x128_P4 = 7, GEMM_DIRECT = 8, GEMM_DIRECT_K2 = 9, GEMM_DIRECT_K4 = 10,
    kGemmTiles = 11
};
bool gemm_tile_valid(int tile, int64_t N);
inline bool gemm_tile_direct(int tile) {
    return tile == GEMM_DIRECT || tile == GEMM_DIRECT_K2 || tile == GEMM_DIRECT_K4;
}
// tile usable for forward layer l of output width N and input width K
bool gemm_tile_valid_layer(int tile, int l, int64_t N, int64_t K);

// C = A B^T with an epilogue; tile < 0 picks a default for the shape.
int32_t launch_gemm(hipStream_t st, int epi, const uint16_t* A, int lda, const uint16_t* B, int ldb, int64_t M,
                    int64_t N, int64_t K, const float* bias, void* C, int ldc, const uint16_t* mask, int tile = -1);

}  // namespace pcfr

struct pcfr_leafnet {
    pcfr::LeafNetPlan P;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    int64_t adam_t = 0;
    std::vector<int> fwd_tile;            // per forward layer GEMM tile, -1 = default
};

namespace pcfr {

// Optional per-launch timing: events recorded around every launch, tagged
// with a kernel class (0 bookkeeping, 1 forward, 2 terminal, 3 backward,
// 4 leaves, 5 hidden-layer GEMMs, 6 output-layer GEMM).
struct LaunchTimer {
    std::vector<hipEvent_t> ev;
    std::vector<int> cls, tag;   // per timed launch: cost class, and a caller tag (-1 if none)
    hipStream_t stream;
    void before(int c, int t = -1) {
        hipEvent_t a;
        (void)hipEventCreate(&a);
        (void)hipEventRecord(a, stream);
        ev.push_back(a);
        cls.push_back(c);
        tag.push_back(t);
    }
    void after() {
        hipEvent_t b;
        (void)hipEventCreate(&b);
        (void)hipEventRecord(b, stream);
        ev.push_back(b);
    }
};

// allow_direct = false runs every layer with a row-major LDS-staged tile
// (training needs row-major activations for its backward pass)
int32_t leafnet_forward_staged(pcfr_leafnet* n, int64_t M, hipStream_t st, LaunchTimer* tm = nullptr,
                               bool allow_direct = true);
int32_t leafnet_autotune(pcfr_leafnet* n, int64_t M, int reps, double* ms_before, double* ms_after);
}
