// run_chains for callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation).
//
// run_chains keeps its launch table (one StepItem per 64-chain group) in a
// library workspace that grows with hipMalloc and is filled from pinned host
// memory.  This variant keeps the table in `scratch`, a file-scope device
// array of fixed size that every GPU the library runs on holds until the
// process ends, and fills it on the device from one item passed by value, so
// the call makes no allocation and no host-to-device copy.  The array's device
// address comes from hipGetSymbolAddress, once per device; kernels only ever
// receive that address.
//
// Limits: at most kNoAllocItems 64-chain groups per call; networks whose
// lane-per-chain rows need device scratch beyond LDS (n > 10240 with k > 6)
// are refused; the node-split form is never used.  Every call on one GPU
// shares that GPU's array, so calls that overlap on one GPU (different
// streams or threads) race and must be serialised by the caller.
#include <mutex>

#include "pbn_driver.h"

namespace pbn {

// 4096 groups of 64 chains: 262144 chains per call.
constexpr uint32_t kNoAllocItems = 4096;
constexpr size_t kNoAllocBytes = (size_t)kNoAllocItems * sizeof(StepItem);
static_assert(PBN_NOALLOC_MAX_CHAINS == 64u * kNoAllocItems, "header limit");
static_assert(kNoAllocBytes == 384u * 1024u, "header size");

static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace {

// Item g of the table: the prototype with chains [64 g, min(64 g + 64, omega)).
__global__ void __launch_bounds__(256) k_fill_items(StepItem *__restrict__ table, StepItem proto, uint32_t omega,
                                                    uint32_t count)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= count) return;
    StepItem it = proto;
    it.chain0 = 64u * g;
    it.nchains = min(64u, omega - 64u * g);
    table[g] = it;
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
StepItem *g_table[kMaxDevices] = {};

// The device address of this device's `scratch`, looked up once per device
// (the device must be current).
int scratch_table(int dev, StepItem **out, std::string &err)
{
    if (dev < 0 || dev >= kMaxDevices) {
        err = "device index beyond the library's table";
        return PBN_ELIMIT;
    }
    std::lock_guard<std::mutex> hold(g_mu);
    if (!g_table[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return PBN_EDEVICE;
        }
        g_table[dev] = (StepItem *)ptr;
    }
    *out = g_table[dev];
    return PBN_OK;
}

}  // namespace

int run_chains_noalloc_impl(pbn_sim *sim, uint64_t burn_in, uint64_t steps, uint32_t thin, std::string &err)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "hipGetDevice";
        return PBN_EDEVICE;
    }
    if (dev != sim->device) {
        err = "the current device is not the simulation's";
        return PBN_EINVAL;
    }
    const uint32_t groups = (sim->omega + 63) / 64;
    if (groups > kNoAllocItems) {
        err = "more than PBN_NOALLOC_MAX_CHAINS chains for the allocation-free call";
        return PBN_ELIMIT;
    }
    StepItem proto{};
    proto.sim = sim->d_desc;
    proto.t0 = (uint32_t)sim->t_done;
    proto.nburn = (uint32_t)burn_in;
    proto.nrec = (uint32_t)steps;
    proto.thin = thin;
    proto.pos0 = sim->len;
    proto.nodes = sim->net.n;
    proto.ops_per_step = (float)sim->net.ops_per_step;
    proto.philox_per_step = (float)sim->net.philox_per_step;
    choose_kernel(sim, proto, latency_waves(sim) <= kLatencyWaves ? kShapeLatency : kShapeAlone);
    if (proto.kernel == 0 && step_rows_words(groups, sim->net.W) > 0) {
        err = "state rows beyond LDS need device scratch: not available without allocation";
        return PBN_ELIMIT;
    }
    StepItem *table = nullptr;
    int rc = scratch_table(dev, &table, err);
    if (rc) return rc;
    if (burn_in + steps * thin > 0) {
        hipLaunchKernelGGL(k_fill_items, dim3((groups + 255) / 256), dim3(256), 0, sim->stream, table, proto,
                           sim->omega, groups);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            err = std::string("k_fill_items launch: ") + hipGetErrorString(e);
            return PBN_EDEVICE;
        }
        rc = proto.kernel == 0
                 ? launch_step(table, groups, sim->net.W, nullptr, sim->stream, err)
                 : launch_step_bs(table, groups, proto.kernel, proto.small != 0, proto.lds, sim->stream, err);
        if (rc) return rc;
    }
    sim->t_done += burn_in + steps * thin;
    sim->len += steps;
    return PBN_OK;
}

}  // namespace pbn
