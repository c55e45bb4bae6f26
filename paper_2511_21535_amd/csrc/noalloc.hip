// p2p_eval_gravity_noalloc: the near-field gravity evaluation for callers that
// cannot allocate device memory.  The only scratch the evaluation needs is the
// GATHER layout's box-sorted rows (x, y, z, m), one 32-byte row per particle;
// here they live in a file-scope device array of fixed size instead of a
// caller workspace.  Each GPU the library runs on holds its own copy of the
// array, at its own address, until the process ends.
#include <mutex>

#include "p2p_internal.h"

namespace p2p {
namespace {

// Rows of the static scratch: 2^21 particles, 64 MiB per GPU.
constexpr int64_t kNoAllocRows = int64_t(1) << 21;
constexpr int kNoAllocDevices = 64;

}  // namespace
}  // namespace p2p

// Host code must not pass this name to a kernel: on the host it is a stand-in,
// not a device address.  Its address on each device comes from
// hipGetSymbolAddress (scratch_rows below).
static __device__ __align__(256) p2p::Row4d scratch[p2p::kNoAllocRows];

namespace p2p {
namespace {

std::mutex g_scratch_mu;
Row4d *g_scratch_ptr[kNoAllocDevices] = {};

// The address of the current device's copy of `scratch`, looked up once per
// device on the first call made with that device current.
p2p_status scratch_rows(Row4d **out) {
    int dev = -1;
    P2P_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocDevices)
        return fail(P2P_EUNSUPPORTED, "device ordinal " + std::to_string(dev) + " beyond the " +
                                          std::to_string(kNoAllocDevices) + " devices the static scratch serves");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(P2P_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<Row4d *>(p);
    }
    *out = g_scratch_ptr[dev];
    return P2P_OK;
}

}  // namespace
}  // namespace p2p

using namespace p2p;

extern "C" p2p_status p2p_eval_gravity_noalloc(const p2p_tree *tree, const p2p_nbrs *nbrs,
                                               const p2p_redundant *red, p2p_layout layout,
                                               p2p_precision prec, double eps, const double *x,
                                               const double *y, const double *z, const double *m,
                                               double *phi, double *ax, double *ay, double *az,
                                               p2p_stream_t stream) {
    set_error("");
    P2P_TRY(gravity_check_args(tree, nbrs, layout, prec, eps));
    Row4d *rows = nullptr;
    if (layout == P2P_GATHER) {
        if (tree->n > kNoAllocRows)
            return fail(P2P_EUNSUPPORTED, "tree->n = " + std::to_string(tree->n) + " exceeds the " +
                                              std::to_string(kNoAllocRows) +
                                              " rows of the static scratch; use p2p_eval_gravity with a workspace");
        P2P_TRY(scratch_rows(&rows));
    }
    // every scratch row the kernels read is written first by this call (the
    // scatter of x, y, z, m into box order), so nothing needs clearing
    return gravity_run(tree, nbrs, red, layout, prec, eps, x, y, z, m, phi, ax, ay, az, rows,
                       static_cast<hipStream_t>(stream));
}
