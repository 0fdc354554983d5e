// Dominance test of online pruning on the GPU (Sec. 5, online pruning):
// before the iterations start, an action whose optimistic value is below the
// pessimistic value of one of its siblings is dominated; the decisions at the
// information sets are independent, so the pass is one workgroup per public
// decision node with its threads spread over the private hands.
//
// A public tree computes all hands of a node together, so removing an action
// for a subset of the hands saves no work; the library removes an action from
// the tree when it is dominated for every hand of the actor's range that the
// node's board does not block (prune_tree then drops its subtree).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "host.hpp"

namespace pcfr {
namespace {

struct PruneNode {
    int32_t first_child, n_child, player, pad;
    uint64_t board;   // every public card at the node
};

constexpr int kPruneBlock = 256;
static_assert(kMaxActions < 31, "one mask bit per action plus the examined bit");

// For a hand h of the actor's range not blocked by the node's board, action
// a is dominated when hi[a][h] < max over b != a of lo[b][h]: the largest
// lower bound among the siblings, which is the largest overall unless a holds
// it, then the second largest.  Each thread ORs into the workgroup's mask bit
// a for every hand where a is not dominated, and bit 31 once it has examined
// a hand; an action is removed when some hand was examined and none left it
// undominated.  A NaN lower bound dominates nothing (it never enters the
// maxima); a NaN upper bound is never dominated.
__global__ __launch_bounds__(kPruneBlock) void k_prune_dominated(const PruneNode* __restrict__ nodes,
                                                                 const uint64_t* __restrict__ combo_mask,
                                                                 const double* __restrict__ ranges,
                                                                 const double* __restrict__ lo,
                                                                 const double* __restrict__ hi,
                                                                 uint8_t* __restrict__ removed) {
    __shared__ uint32_t keep;
    const PruneNode nd = nodes[blockIdx.x];
    if (threadIdx.x == 0) keep = 0;
    __syncthreads();
    uint32_t mine = 0;
    const double* rp = ranges + (size_t)nd.player * kCombos;
    for (int k = threadIdx.x; k < kCombos; k += kPruneBlock) {
        if (!(rp[k] > 0.0) || (combo_mask[k] & nd.board)) continue;
        mine |= 1u << 31;
        double m1 = -INFINITY, m2 = -INFINITY;
        int i1 = -1;
        for (int b = 0; b < nd.n_child; b++) {
            const double x = lo[(size_t)(nd.first_child + b) * kCombos + k];
            if (x > m1) { m2 = m1; m1 = x; i1 = b; }
            else if (x > m2) m2 = x;
        }
        for (int a = 0; a < nd.n_child; a++) {
            const double other = a == i1 ? m2 : m1;
            if (!(hi[(size_t)(nd.first_child + a) * kCombos + k] < other)) mine |= 1u << a;
        }
    }
    if (mine) atomicOr(&keep, mine);
    __syncthreads();
    if ((int)threadIdx.x < nd.n_child)
        removed[nd.first_child + threadIdx.x] = (uint8_t)((keep >> 31) && !(keep >> threadIdx.x & 1u));
}

int32_t hip_fail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return PCFR_E_DEVICE;
}

bool on_device(const void* p) {
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

// Host half shared by both entry points: validate the arguments and list
// the decision nodes and each combo's card mask.
int32_t prune_inputs(const pcfr_tree* tree, const double* ranges, const double* lo, const double* hi,
                     uint8_t* removed, std::vector<PruneNode>& dec, std::vector<uint64_t>& cm) {
    if (!tree || !ranges || !lo || !hi || !removed) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    if (!on_device(lo) || !on_device(hi)) { set_error("the bounds must be device memory"); return PCFR_E_INVALID_ARG; }
    for (int i = 0; i < 2 * kCombos; i++)
        if (!(ranges[i] >= 0.0) || !std::isfinite(ranges[i])) { set_error("ranges must be finite and >= 0"); return PCFR_E_INVALID_ARG; }
    const Tree& t = tree->t;
    try {
        for (const Node& n : t.nodes)
            if (n.type == PCFR_NODE_DECISION) dec.push_back(PruneNode{n.first_child, n.n_child, n.player, 0, n.board_mask});
        cm.resize(kCombos);
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return PCFR_E_OUT_OF_MEMORY;
    }
    const ComboTable& cc = combos();
    for (int k = 0; k < kCombos; k++) cm[k] = (1ull << cc.hi[k]) | (1ull << cc.lo[k]);
    std::memset(removed, 0, t.nodes.size());
    return PCFR_OK;
}

__global__ void k_zero_u8(uint8_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// Device scratch of the allocation-free entry point, one copy per GPU for
// the life of the process: the decision-node list, the combo masks, the
// ranges and the per-node flags.  Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr int64_t kScratchDecisions = 65536;
constexpr int64_t kScratchNodes = 262144;
constexpr size_t kScrNodesOff = 0;
constexpr size_t kScrMaskOff = kScrNodesOff + sizeof(PruneNode) * kScratchDecisions;
constexpr size_t kScrRangeOff = kScrMaskOff + sizeof(uint64_t) * kCombos;
constexpr size_t kScrFlagOff = kScrRangeOff + sizeof(double) * 2 * kCombos;
constexpr size_t kScratchBytes = kScrFlagOff + kScratchNodes;
static_assert(kScrMaskOff % 16 == 0 && kScrRangeOff % 16 == 0 && kScrFlagOff % 16 == 0, "aligned sections");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of scratch (looked up once per device).
int32_t scratch_for_current_device(unsigned char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) { set_error("device index beyond the scratch table"); return PCFR_E_DEVICE; }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return hip_fail(e, "hipGetSymbolAddress");
        if (!p) { set_error("hipGetSymbolAddress returned no address"); return PCFR_E_DEVICE; }
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return PCFR_OK;
}

}  // namespace
}  // namespace pcfr

using namespace pcfr;

extern "C" int32_t pcfr_prune_dominated(const pcfr_tree* tree, const double* ranges, const double* lo,
                                        const double* hi, uint8_t* removed) {
    std::vector<PruneNode> dec;
    std::vector<uint64_t> cm;
    int32_t rc = prune_inputs(tree, ranges, lo, hi, removed, dec, cm);
    if (rc != PCFR_OK) return rc;
    const size_t N = tree->t.nodes.size();
    if (dec.empty()) return PCFR_OK;
    DevBuf dn, dm, dr, dout;
    hipError_t e;
    if ((e = hipMalloc(&dn.p, sizeof(PruneNode) * dec.size())) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = hipMalloc(&dm.p, sizeof(uint64_t) * kCombos)) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = hipMalloc(&dr.p, sizeof(double) * 2 * kCombos)) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = hipMalloc(&dout.p, N)) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = hipMemcpy(dn.p, dec.data(), sizeof(PruneNode) * dec.size(), hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
    if ((e = hipMemcpy(dm.p, cm.data(), sizeof(uint64_t) * kCombos, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
    if ((e = hipMemcpy(dr.p, ranges, sizeof(double) * 2 * kCombos, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
    if ((e = hipMemset(dout.p, 0, N)) != hipSuccess) return hip_fail(e, "hipMemset");
    hipLaunchKernelGGL(k_prune_dominated, dim3((unsigned)dec.size()), dim3(kPruneBlock), 0, 0,
                       (const PruneNode*)dn.p, (const uint64_t*)dm.p, (const double*)dr.p, lo, hi, (uint8_t*)dout.p);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_prune_dominated");
    if ((e = hipMemcpy(removed, dout.p, N, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "hipMemcpy");
    return PCFR_OK;
}

extern "C" int32_t pcfr_prune_dominated_noalloc(const pcfr_tree* tree, const double* ranges, const double* lo,
                                                const double* hi, uint8_t* removed) {
    std::vector<PruneNode> dec;
    std::vector<uint64_t> cm;
    int32_t rc = prune_inputs(tree, ranges, lo, hi, removed, dec, cm);
    if (rc != PCFR_OK) return rc;
    const int64_t N = (int64_t)tree->t.nodes.size();
    if ((int64_t)dec.size() > kScratchDecisions || N > kScratchNodes) {
        set_error("tree exceeds the static scratch of pcfr_prune_dominated_noalloc (65536 decision nodes, "
                  "262144 nodes)");
        return PCFR_E_TOO_LARGE;
    }
    if (dec.empty()) return PCFR_OK;
    unsigned char* base = nullptr;
    if ((rc = scratch_for_current_device(&base)) != PCFR_OK) return rc;
    PruneNode* dn = reinterpret_cast<PruneNode*>(base + kScrNodesOff);
    uint64_t* dm = reinterpret_cast<uint64_t*>(base + kScrMaskOff);
    double* dr = reinterpret_cast<double*>(base + kScrRangeOff);
    uint8_t* dout = base + kScrFlagOff;
    hipError_t e;
    if ((e = hipMemcpy(dn, dec.data(), sizeof(PruneNode) * dec.size(), hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
    if ((e = hipMemcpy(dm, cm.data(), sizeof(uint64_t) * kCombos, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
    if ((e = hipMemcpy(dr, ranges, sizeof(double) * 2 * kCombos, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
    // the flags of the previous call are still there: clear this call's span
    const unsigned zb = (unsigned)std::min<int64_t>((N + 255) / 256, 1024);
    hipLaunchKernelGGL(k_zero_u8, dim3(zb), dim3(256), 0, 0, dout, N);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_zero_u8");
    hipLaunchKernelGGL(k_prune_dominated, dim3((unsigned)dec.size()), dim3(kPruneBlock), 0, 0,
                       (const PruneNode*)dn, (const uint64_t*)dm, (const double*)dr, lo, hi, dout);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_prune_dominated");
    if ((e = hipMemcpy(removed, dout, (size_t)N, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "hipMemcpy");
    return PCFR_OK;
}
