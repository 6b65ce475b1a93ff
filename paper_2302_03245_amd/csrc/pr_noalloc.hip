// pr_noalloc.hip -- pr_solve_ifp2_noalloc: IFP2 (Algorithm 3) with its whole solve
// workspace taken from a fixed device array instead of allocated memory, for callers
// that cannot allocate (stream capture, serving loops, harnesses that forbid it).
#include "pr_host.h"

namespace prk {
namespace {

// Workspace of every pr_solve_ifp2_noalloc call on a device: one array per device
// (each GPU the library runs on holds its own copy until the process ends).  Calls
// that overlap on one device share it and race.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's array (hipGetSymbolAddress once per device, with
// that device current); in host code the array's own name is not a device address.
pr_status scratch_of(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return host::fail(PR_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return host::hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PR_OK;
}

}  // namespace
}  // namespace prk

using namespace prk;
using namespace prk::host;

extern "C" {

pr_status pr_solve_ifp2_noalloc(const pr_graph *g, const double *p, const pr_opts *o, double *pi, pr_stats *st) {
    g_err.clear();
    if (!g) return fail(PR_EINVAL, "graph is NULL");
    if (!pi) return fail(PR_EINVAL, "pi is NULL");
    pr_opts op;
    opts_or_default(o, &op);
    pr_status ps = check_opts(op, false);
    if (ps != PR_OK) return ps;
    if (op.flags & PR_PROFILE) return fail(PR_EINVAL, "PR_PROFILE times kernels with events: not without allocation");
    ps = enter(g);
    if (ps != PR_OK) return ps;
    const Graph &G = g->g;
    const size_t need = op.residual == PR_RES_FP32 ? solve_ifp_bytes<float>(G, true, p, op, false)
                                                   : solve_ifp_bytes<double>(G, true, p, op, false);
    if (need > kScratchBytes)
        return fail(PR_EINVAL, "this solve needs " + std::to_string(need) + " bytes of workspace; " +
                                   "pr_solve_ifp2_noalloc has " + std::to_string(kScratchBytes));
    void *base = nullptr;
    ps = scratch_of(G.device, &base);
    if (ps != PR_OK) return ps;
    GraphUse use;
    ps = use_graph(G, use);
    if (ps != PR_OK) return ps;
    Ctl hctl;  // host copy of the control block (pageable)
    ExtWorkspace ext{base, kScratchBytes, &hctl};
    try {
        return op.residual == PR_RES_FP32 ? solve_ifp_t<float>(G, true, p, -1, op, pi, st, nullptr, &ext)
                                          : solve_ifp_t<double>(G, true, p, -1, op, pi, st, nullptr, &ext);
    } catch (const std::bad_alloc &) {
        return fail(PR_ENOMEM, "host allocation");
    }
}

}  // extern "C"
