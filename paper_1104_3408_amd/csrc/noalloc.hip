// Constraint monitor that allocates nothing: ghg_constraints_static.
//
// ghg_constraints reduces its constraint fields through workgroup partials
// in a workspace the grid allocates, and computes the Cartesian derivatives
// of g_ab into the grid's derivative workspace.  This variant takes the
// derivatives from the caller (the layout spec_derivs writes in SG_CART
// mode) and keeps the partials in a fixed device array of this file, so a
// call makes no allocation of any kind: for callers that cannot allocate
// device memory (code being captured into a graph, serving loops, harnesses
// that forbid it).
#include <mutex>

#include "internal.h"

// Workgroup partials (4 doubles per 256 grid points of one shell): 4096
// workgroups cover 1,048,576 points per shell, more than the largest shell
// shell_grid_create accepts (80 x 64 x 128).  128 KB on every device the
// library runs on, held until the process ends.
constexpr int kScratchParts = 4096;
static __device__ __align__(256) double scratch[4 * kScratchParts];

namespace sg {

namespace {

// Device address of this device's copy of scratch, looked up once per device
// with that device current (in host code the array's name is only a host
// stand-in, never a device address).
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

hipError_t scratch_address(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

}  // namespace sg

using namespace sg;

extern "C" sg_status ghg_constraints_static(const sg_grid* g, const double* u, const double* du_cart, double* norms,
                                            sg_stream_t stream) {
    if (!g || !u || !du_cart || !norms) return set_error(SG_EINVAL, "NULL argument");
    for (const ShellHost& S : g->sh)
        if ((S.npts + 255) / 256 > (size_t)kScratchParts)
            return set_error(SG_ESHAPE, "ghg_constraints_static: a shell has more than 4096 x 256 grid points");
    double* part = nullptr;
    hipError_t e = scratch_address(&part);
    if (e != hipSuccess) return set_error(SG_EHIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    hipStream_t st = (hipStream_t)stream;
    for (int s = 0; s < (int)g->sh.size(); ++s) {
        const ShellHost& S = g->sh[s];
        const KShell v = S.view(g->opt.n_fields);
        // g_ab's derivatives are the first ten variables of each of the three
        // Cartesian blocks of this shell (each block one shell state long)
        e = launch_constraints(v, u + S.off, du_cart + 3 * S.off, (long long)S.count, part, norms + 4 * s, st);
        if (e != hipSuccess) return set_error(SG_EHIP, std::string("constraint launch: ") + hipGetErrorString(e));
    }
    return SG_OK;
}
