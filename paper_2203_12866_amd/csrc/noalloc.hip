// cosenu_step_noalloc: RK4 steps of a caller-owned device state with every
// intermediate buffer in one static device array, for callers that cannot
// allocate device memory.  It runs the kernels cosenu_step runs (fused stage
// pairs where the shape allows them, else four single stages per step), with
// the default launch shapes; results do not depend on launch shapes, so they
// are those of a handle created from the same parameters, bit for bit.
#include <cstring>
#include <mutex>

#include "cosenu.h"
#include "cosenu_host.h"
#include "cosenu_internal.h"

using namespace cosenu;

namespace {

// The scratch array: a file-scope device array, one copy per GPU, held until
// the process ends.  Host code never uses its name as an address: the device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = COSENU_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (the current device must be dev).
hipError_t scratch_for(int dev, void **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Per-point constants travel to the device as kernel arguments (by value), a
// chunk per launch: no host buffer has to outlive the call.
constexpr int kConstChunk = 240;
struct ConstChunk {
    double v[kConstChunk];
};

__global__ __launch_bounds__(256) void put_constants(double *dst, int n, ConstChunk c) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = c.v[i];
}

// Byte offsets of the buffers inside the scratch array for one problem; the
// total is the scratch it needs.
struct Layout {
    size_t consts, acc, buf1, yb, mom[4], total;
};

Layout layout_for(const InstDesc &d) {
    Layout L;
    const size_t cells = (size_t)d.nz * d.nv;
    size_t at = 0;
    L.consts = at;
    at = align256(at + 4 * (size_t)d.nv * sizeof(double));
    L.acc = at;
    at = align256(at + 8 * cells * sizeof(double));
    L.buf1 = at;  // Y2 / Y4, or the second state buffer of the fused pairs
    at = align256(at + 8 * cells * sizeof(double));
    L.yb = at;
    at = align256(at + 8 * cells * (d.form == COSENU_FP64 ? sizeof(double) : sizeof(float)));
    const size_t mom = (size_t)d.nz * d.vchunks * 2 * kMomQ * sizeof(double);
    for (int k = 0; k < 4; ++k) {
        L.mom[k] = at;
        at = align256(at + mom);
    }
    L.total = at;
    return L;
}

}  // namespace

extern "C" int cosenu_step_noalloc(const cosenu_params *p, double *state, int64_t nsteps, void *hip_stream) try {
    if (!p || !state || nsteps < 0) return COSENU_EINVAL;
    char why[256];
    if (params_problem(*p, why, sizeof why)) return COSENU_EINVAL;
    InstDesc d;
    fill_desc_constants(*p, d);
    d.ps = (size_t)p->nz * p->nv;  // the caller's [8][nz][nv] layout, planes unpadded
    const Layout L = layout_for(d);
    if (L.total > kScratchBytes) return COSENU_EINVAL;
    if (nsteps == 0) return COSENU_OK;
    const hipStream_t st = (hipStream_t)hip_stream;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return COSENU_EDEVICE;
    void *base = nullptr;
    if (scratch_for(dev, &base) != hipSuccess) return COSENU_EDEVICE;
    char *b = (char *)base;
    double *consts = (double *)(b + L.consts);
    d.vel = consts;
    d.g = consts + d.nv;
    d.gb = consts + 2 * d.nv;
    d.agb = consts + 3 * d.nv;
    d.acc = (double *)(b + L.acc);
    double *buf[2] = {state, (double *)(b + L.buf1)};
    d.y = buf[0];
    d.ya = buf[1];
    d.yb = b + L.yb;
    for (int k = 0; k < 4; ++k) d.mom[k] = (double *)(b + L.mom[k]);
    // default launch shapes (the tuning cache is not consulted: reading it
    // allocates on the host); results do not depend on launch shapes
    const bool pairs = pair_supported(d);

    // per-point constants, every element computed as the handle's table is
    const double s_nu = gaussian_norm(p->nv, p->quadrature, p->sigma_nu);
    const double s_nubar = gaussian_norm(p->nv, p->quadrature, p->sigma_nubar);
    const int nconst = 4 * p->nv;
    for (int k0 = 0; k0 < nconst; k0 += kConstChunk) {
        ConstChunk c;
        const int n = nconst - k0 < kConstChunk ? nconst - k0 : kConstChunk;
        for (int i = 0; i < n; ++i) c.v[i] = bin_constant_at(*p, k0 + i, s_nu, s_nubar);
        for (int i = n; i < kConstChunk; ++i) c.v[i] = 0.0;
        hipLaunchKernelGGL(put_constants, dim3(1), dim3(256), 0, st, consts + k0, n, c);
        if (hipGetLastError() != hipSuccess) return COSENU_EDEVICE;
    }
    // moments of the stage-1 input: the caller's state may be new
    if (launch_moments_init(d, blocks_for(d), st) != hipSuccess) return COSENU_EDEVICE;
    int par = 0;
    for (int64_t k = 0; k < nsteps; ++k) {
        if (pairs) {
            d.y = buf[par];
            d.ya = buf[par ^ 1];
            if (launch_pair(d, 0, st) != hipSuccess || launch_pair(d, 1, st) != hipSuccess) return COSENU_EDEVICE;
            par ^= 1;
        } else {
            for (int s = 0; s < 4; ++s)
                if (launch_stage(d, s, blocks_for(d), st) != hipSuccess) return COSENU_EDEVICE;
        }
    }
    // an odd number of fused steps leaves the state in the second buffer
    if (par == 1 && hipMemcpyAsync(state, buf[1], 8 * d.ps * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return COSENU_EDEVICE;
    return COSENU_OK;
} COSENU_ABI_CATCH(nullptr)
