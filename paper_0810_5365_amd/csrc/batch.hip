// Persistent batch: the even-odd hopping term of several lattices of uneven
// volume, each with its own number of right-hand sides, in ONE kernel launch
// captured in a hipGraph.
//
// The work list is a sequence of tiles (item, rhs, block of W output sites,
// W the workgroup size), rhs-innermost so that the tiles sharing one block of
// links are adjacent.  The grid is sized to the device (a few waves per
// compute unit); after the XCD-aware remap, logical workgroup b owns the
// contiguous tile range [N b / G, N (b+1) / G), so each XCD walks one
// contiguous stretch of the list and every workgroup runs a bounded loop with
// no waits.  The tile width, the waves per compute unit and the software
// pipelining of the directions are autotuned when the batch is created.
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "dslash_body.h"

namespace wd {


struct BatchItem {
    DslashArgs A;
    int dagger;
    int nrhs;
    long long tile0;   // first tile of this item in the global list
};

template <int P, int R, bool NT, bool PF>
__global__ void __launch_bounds__(256) batch_kernel(const BatchItem* __restrict__ items, int nitems, long long ntiles)
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
        const uint32_t cb = (uint32_t)(local / B.nrhs) * blockDim.x + threadIdx.x;
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
    int block = 256, waves_per_cu = 24, pf = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // each item's gauge and whether its links were in temporal gauge when the launch was
    // captured (the kernel skips the unit t-links then); a later upload or fix changes that
    std::vector<std::pair<wd_gauge, bool>> gauge_state;
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

// launch shape of a batch: tile width (= workgroup size), persistent waves per compute unit,
// software-pipelined directions
struct BatchShape {
    int block, wpc;
    bool pf;
};

// tile offsets of the items for tile width `block`; the total tile count
static long long set_tiles(std::vector<BatchItem>& h, int block)
{
    long long ntiles = 0;
    for (BatchItem& B : h) {
        B.tile0 = ntiles;
        ntiles += (long long)((B.A.g.Vh + block - 1) / block) * B.nrhs;
    }
    return ntiles;
}

static int batch_grid(long long ntiles, int cus, const BatchShape& sh)
{
    const long long cap = (long long)cus * sh.wpc * 64 / sh.block;
    return (int)(ntiles < cap ? ntiles : cap);
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
    }
    hipDeviceProp_t prop;
    WD_HIP(hipGetDeviceProperties(&prop, ctx->device));
    const int cus = prop.multiProcessorCount;

    wd_batch b = new wd_batch_s();
    b->ctx = ctx;
    b->nitems = n;
    for (int i = 0; i < n; ++i) b->gauge_state.emplace_back(items[i].gauge, items[i].gauge->gf);
    auto fail = [&](wd_status s) {
        destroy_batch(b);
        return s;
    };
    if (hipMalloc(&b->ditems, sizeof(BatchItem) * n) != hipSuccess) {
        set_error("wd_batch_create: device allocation failed");
        return fail(WD_ENOMEM);
    }
    // the launch shape: forced by WD_BATCH_BLOCK / WD_BATCH_WAVES / WD_BATCH_PF if any is set,
    // else the fastest of the candidates, each timed on the batch itself (three launches after
    // one warm-up, the minimum), unless WD_BATCH_TUNE=0 (then 256-site tiles, 24 waves per CU)
    BatchShape best{256, 24, false};
    const char* eb = getenv("WD_BATCH_BLOCK");
    const char* ew = getenv("WD_BATCH_WAVES");
    const char* ep = getenv("WD_BATCH_PF");
    const char* et = getenv("WD_BATCH_TUNE");
    if (eb || ew || ep) {
        if (eb) best.block = atoi(eb);
        if (ew) best.wpc = atoi(ew);
        if (ep) best.pf = atoi(ep) != 0;
        if (best.block < 64 || best.block > 256 || best.block % 64 || best.wpc < 1 || best.wpc > 64) {
            set_error("wd_batch_create: WD_BATCH_BLOCK must be 64..256 in steps of 64, WD_BATCH_WAVES 1..64");
            return fail(WD_EINVAL);
        }
    } else if (!(et && atoi(et) == 0)) {
        float best_us = 1e30f;
        for (int block : {64, 128, 256})
            for (int wpc : {8, 16, 24, 32})
                for (int pf = 0; pf < 2; ++pf) {
                    const BatchShape sh{block, wpc, pf != 0};
                    const long long nt = set_tiles(h, block);
                    if (hipMemcpy(b->ditems, h.data(), sizeof(BatchItem) * n, hipMemcpyHostToDevice) != hipSuccess) {
                        set_error("wd_batch_create: HIP copy failed");
                        return fail(WD_EHIP);
                    }
                    void* kern = pick_batch_kernel(prec, recon, sh.pf);
                    const BatchItem* di = b->ditems;
                    int ni = n;
                    long long ntv = nt;
                    void* args[] = {(void*)&di, (void*)&ni, (void*)&ntv};
                    const int grid = batch_grid(nt, cus, sh);
                    float ms = 0.f;
                    hipError_t e = hipLaunchKernel(kern, dim3(grid), dim3(block), args, 0, ctx->stream);
                    if (e == hipSuccess) e = hipEventRecord(ctx->ev0, ctx->stream);
                    for (int r = 0; r < 3 && e == hipSuccess; ++r)
                        e = hipLaunchKernel(kern, dim3(grid), dim3(block), args, 0, ctx->stream);
                    if (e == hipSuccess) e = hipEventRecord(ctx->ev1, ctx->stream);
                    if (e == hipSuccess) e = hipEventSynchronize(ctx->ev1);
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
                    if (e != hipSuccess) {
                        set_error("wd_batch_create: timing a launch shape failed: %s", hipGetErrorString(e));
                        return fail(WD_EHIP);
                    }
                    if (ms / 3 * 1000.f < best_us) {
                        best_us = ms / 3 * 1000.f;
                        best = sh;
                    }
                }
    }
    const long long ntiles = set_tiles(h, best.block);
    const int grid = batch_grid(ntiles, cus, best);
    void* kern = pick_batch_kernel(prec, recon, best.pf);
    b->ntiles = ntiles;
    b->grid = grid;
    b->block = best.block;
    b->waves_per_cu = best.wpc;
    b->pf = best.pf ? 1 : 0;
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
    hipError_t le = hipLaunchKernel(kern, dim3(grid), dim3(best.block), args, 0, b->cap);
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
    for (size_t i = 0; i < b->gauge_state.size(); ++i)
        if (b->gauge_state[i].first->gf != b->gauge_state[i].second) {
            set_error("wd_batch_run: item %zu's gauge was %s since the batch was created; create the batch again",
                      i, b->gauge_state[i].second ? "uploaded again" : "fixed to the temporal gauge");
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

wd_status wd_batch_shape(wd_batch b, int* block, int* waves_per_cu, int* pf)
{
    if (!b || !block || !waves_per_cu || !pf) {
        set_error("wd_batch_shape: NULL argument");
        return WD_EINVAL;
    }
    *block = b->block;
    *waves_per_cu = b->waves_per_cu;
    *pf = b->pf;
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
