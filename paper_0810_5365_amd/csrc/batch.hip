// Persistent batch: the even-odd hopping term of several lattices of uneven
// volume, each with its own number of right-hand sides, in ONE kernel launch
// captured in a hipGraph.
//
// The work list is a sequence of tiles (item, rhs, block of 256 output
// sites), rhs-innermost so that the tiles sharing one block of links are
// adjacent.  The grid is sized to the device (a few workgroups per compute
// unit); after the XCD-aware remap, logical workgroup b owns the contiguous
// tile range [N b / G, N (b+1) / G), so each XCD walks one contiguous stretch
// of the list and every workgroup runs a bounded loop with no waits.
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "dslash_body.h"

namespace wd {

constexpr int BATCH_BLOCK = 256;

struct BatchItem {
    DslashArgs A;
    int dagger;
    int nrhs;
    long long tile0;   // first tile of this item in the global list
};

template <int P, int R, bool NT, bool PF>
__global__ void __launch_bounds__(BATCH_BLOCK) batch_kernel(const BatchItem* __restrict__ items, int nitems,
                                                            long long ntiles)
{
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const long long t0 = ntiles * lb / gridDim.x;
    const long long t1 = ntiles * (lb + 1) / gridDim.x;
    int it = 0;
    for (long long t = t0; t < t1; ++t) {
        while (it + 1 < nitems && items[it + 1].tile0 <= t) ++it;
        const BatchItem& B = items[it];
        const long long local = t - B.tile0;
        const int rhs = (int)(local % B.nrhs);
        const uint32_t cb = (uint32_t)(local / B.nrhs) * BATCH_BLOCK + threadIdx.x;
        if (cb < (uint32_t)B.A.g.Vh) {
            if (B.dagger) dslash_site<P, R, true, false, NT, PF>(B.A, cb, rhs);
            else dslash_site<P, R, false, false, NT, PF>(B.A, cb, rhs);
        }
    }
}

} // namespace wd

struct wd_batch_s {
    wd_context ctx = nullptr;
    wd::BatchItem* ditems = nullptr;
    int nitems = 0;
    long long ntiles = 0;
    int grid = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace wd {

template <int P, int R>
static void* batch_kernel_ptr(bool pf)
{
    return pf ? (void*)batch_kernel<P, R, false, true> : (void*)batch_kernel<P, R, false, false>;
}

static void* pick_batch_kernel(int prec, int recon, bool pf)
{
    const bool r12 = recon == 12;
    switch (prec) {
    case WD_F64: return r12 ? batch_kernel_ptr<P_F64, 12>(pf) : batch_kernel_ptr<P_F64, 18>(pf);
    case WD_F32: return r12 ? batch_kernel_ptr<P_F32, 12>(pf) : batch_kernel_ptr<P_F32, 18>(pf);
    case WD_F16: return r12 ? batch_kernel_ptr<P_F16, 12>(pf) : batch_kernel_ptr<P_F16, 18>(pf);
    case WD_BF16: return r12 ? batch_kernel_ptr<P_BF16, 12>(pf) : batch_kernel_ptr<P_BF16, 18>(pf);
    }
    return nullptr;
}

static void destroy_batch(wd_batch b)
{
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->cap) hipStreamDestroy(b->cap);
    if (b->ditems) hipFree(b->ditems);
    delete b;
}

} // namespace wd

using namespace wd;

extern "C" {

wd_status wd_batch_create(wd_context ctx, int n, const wd_batch_item* items, wd_prec prec, wd_batch* out)
{
    if (!ctx || !items || !out || n < 1) {
        set_error("wd_batch_create: NULL argument or empty batch");
        return WD_EINVAL;
    }
    if (!valid_prec(prec)) {
        set_error("wd_batch_create: bad precision %d", (int)prec);
        return WD_EINVAL;
    }
    std::vector<BatchItem> h(n);
    long long ntiles = 0;
    int recon = 0;
    for (int i = 0; i < n; ++i) {
        const wd_batch_item& it = items[i];
        if (!it.gauge || !it.in || !it.out || it.nrhs < 1 || it.nrhs > 65535 ||
            (it.out_subset != WD_EVEN && it.out_subset != WD_ODD)) {
            set_error("wd_batch_create: item %d: NULL pointer, nrhs out of range or subset not EVEN/ODD", i);
            return WD_EINVAL;
        }
        if (it.gauge->ctx != ctx) {
            set_error("wd_batch_create: item %d belongs to another context", i);
            return WD_EINVAL;
        }
        if (i == 0) recon = it.gauge->recon;
        if (it.gauge->recon != recon) {
            set_error("wd_batch_create: all items must share one link layout (item %d differs)", i);
            return WD_EUNSUPPORTED;
        }
        const void* links = nullptr;
        WD_TRY(gauge_links(it.gauge, prec, &links));
        const Geom& G = it.gauge->geom;
        const long long hb = (long long)half_bytes(G, prec);
        BatchItem& B = h[i];
        memset(&B, 0, sizeof B);
        B.A.gauge = (const char*)links;
        B.A.in = (const char*)it.in;
        B.A.out = (char*)it.out;
        B.A.x = nullptr;
        B.A.in_stride = B.A.out_stride = hb;
        B.A.x_stride = 0;
        B.A.a = 0.0;
        B.A.b = 1.0;
        B.A.g = G;
        B.A.par = it.out_subset == WD_EVEN ? 0 : 1;
        B.A.remap = 0;
        B.A.rhs_inner = 0;
        B.A.zb = 0;
        B.A.gf = it.gauge->gf ? 1 : 0;
        B.dagger = it.dagger != 0;
        B.nrhs = it.nrhs;
        B.tile0 = ntiles;
        ntiles += (long long)((G.Vh + BATCH_BLOCK - 1) / BATCH_BLOCK) * it.nrhs;
    }
    hipDeviceProp_t prop;
    WD_HIP(hipGetDeviceProperties(&prop, ctx->device));
    const long long cap = (long long)prop.multiProcessorCount * 6;
    const int grid = (int)(ntiles < cap ? ntiles : cap);
    void* kern = pick_batch_kernel(prec, recon, getenv("WD_BATCH_PF") ? atoi(getenv("WD_BATCH_PF")) != 0 : false);

    wd_batch b = new wd_batch_s();
    b->ctx = ctx;
    b->nitems = n;
    b->ntiles = ntiles;
    b->grid = grid;
    auto fail = [&](wd_status s) {
        destroy_batch(b);
        return s;
    };
    if (hipMalloc(&b->ditems, sizeof(BatchItem) * n) != hipSuccess) {
        set_error("wd_batch_create: device allocation failed");
        return fail(WD_ENOMEM);
    }
    if (hipMemcpy(b->ditems, h.data(), sizeof(BatchItem) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        set_error("wd_batch_create: HIP setup failed");
        return fail(WD_EHIP);
    }
    // capture the single persistent launch into a graph
    const BatchItem* ditems = b->ditems;
    int nitems = n;
    void* args[] = {(void*)&ditems, (void*)&nitems, (void*)&ntiles};
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        set_error("wd_batch_create: stream capture failed to start");
        return fail(WD_EHIP);
    }
    hipError_t le = hipLaunchKernel(kern, dim3(grid), dim3(BATCH_BLOCK), args, 0, b->cap);
    hipError_t ce = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess || ce != hipSuccess || !b->graph) {
        set_error("wd_batch_create: capture failed: %s / %s", hipGetErrorString(le), hipGetErrorString(ce));
        return fail(WD_EHIP);
    }
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
        set_error("wd_batch_create: graph instantiation failed");
        return fail(WD_EHIP);
    }
    *out = b;
    return WD_OK;
}

wd_status wd_batch_run(wd_batch b)
{
    if (!b) {
        set_error("wd_batch_run: NULL batch");
        return WD_EINVAL;
    }
    WD_HIP(hipGraphLaunch(b->exec, b->ctx->stream));
    return WD_OK;
}

wd_status wd_batch_info(wd_batch b, long long* ntiles, int* grid)
{
    if (!b || !ntiles || !grid) {
        set_error("wd_batch_info: NULL argument");
        return WD_EINVAL;
    }
    *ntiles = b->ntiles;
    *grid = b->grid;
    return WD_OK;
}

wd_status wd_batch_destroy(wd_batch b)
{
    if (!b) {
        set_error("wd_batch_destroy: NULL batch");
        return WD_EINVAL;
    }
    hipStreamSynchronize(b->ctx->stream);
    destroy_batch(b);
    return WD_OK;
}

} // extern "C"
