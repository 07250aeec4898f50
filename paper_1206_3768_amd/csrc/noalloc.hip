// Allocation-free FP64 Chebyshev filter (chfsi_filter_noalloc).
//
// The same filter steps as chfsi_filter in FP64 with one degree for every column (Algorithm 1,
// filtering step: the scaled three-term recurrence), for callers that cannot allocate device
// memory.  The recurrence needs a second n x m block besides the caller's Y and, for split-K
// plans, the partial tiles of each step; both live in one fixed device array of this file instead
// of a handle's workspace.  Nothing here allocates: the array belongs to the code object, and the
// host only looks up its device address once per device.
#include <mutex>

#include "driver.h"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)CHFSI_NOALLOC_SCRATCH_BYTES;
constexpr size_t SCRATCH_ELEMS = SCRATCH_BYTES / sizeof(zd);

// One copy per device, held until the process ends.  In host code this name is not a device
// address: kernels receive the address from hipGetSymbolAddress below.
static __device__ __align__(256) zd scratch[SCRATCH_ELEMS];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
zd* g_scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up on the first call per device.
chfsi_status scratch_address(zd** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return CHFSI_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CHFSI_ERR_DEVICE;
        g_scratch_dev[dev] = (zd*)p;
    }
    *out = g_scratch_dev[dev];
    return CHFSI_SUCCESS;
}

}  // namespace

extern "C" chfsi_status chfsi_filter_noalloc(void* hip_stream, int n, const void* Hv, int ldh, void* Yv, int ldy,
                                             int m, int deg, double a, double b, double mu1)
{
    if (!Hv || !Yv || n <= 0 || m < 0 || ldh < n || ldy < n || deg < 0) return CHFSI_ERR_ARG;
    if (!(mu1 < a) || !(a < b)) return CHFSI_ERR_ARG;
    zd* ws = nullptr;
    const chfsi_status rs = scratch_address(&ws);   // set-up on every call, also when there is no work
    if (rs != CHFSI_SUCCESS) return rs;
    if (m == 0 || deg == 0) return CHFSI_SUCCESS;
    const size_t block = (size_t)n * (size_t)m;
    if (block > SCRATCH_ELEMS) return CHFSI_ERR_TOO_LARGE;

    hipStream_t st = (hipStream_t)hip_stream;
    const zd* H = (const zd*)Hv;
    zd* Y = (zd*)Yv;
    zd* T = ws;   // the second block of the recurrence, leading dimension n
    // split-K partial tiles after T (256-byte aligned); a plan whose partials do not fit the rest
    // falls back to fewer K slices (one slice: no partials at all)
    const size_t poff = (block + 15) / 16 * 16;
    GemmWs gw;
    if (poff < SCRATCH_ELEMS) {
        gw.ws = ws + poff;
        gw.bytes = (SCRATCH_ELEMS - poff) * sizeof(zd);
    }
    double sigma = 0;
    for (int k = 1; k <= deg; ++k) {
        // Y_k in T for odd k, in Y for even k; the output overwrites Y_{k-2} in place
        const zd* yk = (k % 2 == 1) ? Y : T;
        const int ldk = (k % 2 == 1) ? ldy : n;
        zd* yo = (k % 2 == 1) ? T : Y;
        const int ldo = (k % 2 == 1) ? n : ldy;
        const zd* yp = (k == 1) ? yk : yo;   // beta = 0 on the first step
        const int ldp = (k == 1) ? ldk : ldo;
        const FilterStep fs = filter_step_coefficients(k - 1, a, b, mu1, sigma);
        if (launch_filter_step_f64(st, n, m, H, ldh, yk, ldk, yp, ldp, yo, ldo, fs, gw) != 0) return CHFSI_ERR_DEVICE;
    }
    if (deg % 2 == 1 && launch_zlacpy(st, n, m, T, n, Y, ldy) != 0) return CHFSI_ERR_DEVICE;
    return CHFSI_SUCCESS;
}
