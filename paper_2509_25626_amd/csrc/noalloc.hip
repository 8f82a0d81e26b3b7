// The stand-alone radix sort without any allocation, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid it).  Every buffer the sort needs beyond its inputs
// and outputs (the ping-pong pair buffers, the onesweep status words and
// digit counts, the reduce-then-scan matrices) is carved from one file-scope
// device array, `scratch`, which every GPU the library runs on holds from
// module load until the process ends.
//
// Host code never passes `scratch` itself to a kernel (on the host the name
// is only a stand-in for the symbol): when a context is created, its device's
// copy of the array is looked up once with hipGetSymbolAddress and the
// address kept per device; the kernels receive that address.
//
// All calls on one GPU share its array and it keeps the last call's contents:
// everything that must start at zero is cleared by fill kernels on the
// caller's stream at the start of every call, and two calls that overlap on
// one GPU (different streams, or threads) race on the array.
#include <mutex>

#include "cdnasplat.h"
#include "internal.h"
#include "runtime_internal.h"

using namespace cds;

namespace {

// Layout of the scratch array for at most CDS_NOALLOC_MAX_PAIRS pairs and 8
// passes (each part 256-byte aligned).
constexpr int64_t kMaxPairs = CDS_NOALLOC_MAX_PAIRS;
constexpr int64_t kMaxParts = (kMaxPairs + kSortPartition - 1) / kSortPartition;
constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kOffKeys = 0;
constexpr size_t kOffVals = kOffKeys + align256(sizeof(uint64_t) * kMaxPairs);
constexpr size_t kOffStatus = kOffVals + align256(sizeof(uint32_t) * kMaxPairs);
constexpr size_t kOffPartHist = kOffStatus + align256(sizeof(uint32_t) * 256 * kMaxParts * 8);
constexpr size_t kOffBases = kOffPartHist + align256(sizeof(uint32_t) * 256 * kMaxParts);
constexpr size_t kOffHist = kOffBases + align256(sizeof(uint32_t) * 256 * kMaxParts);
constexpr size_t kOffCounters = kOffHist + align256(sizeof(uint32_t) * 256 * 8);
constexpr size_t kOffScanSums = kOffCounters + 256;
constexpr size_t kScanSumsBytes = 4096;
constexpr size_t kOffScanTotal = kOffScanSums + kScanSumsBytes;
constexpr size_t kScratchBytes = kOffScanTotal + 256;
static_assert(kScratchBytes == CDS_NOALLOC_SCRATCH_BYTES, "the header states the scratch size");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
hipError_t g_status[kMaxDevices] = {};

}  // namespace

namespace cds {

// Called by cds_create with `device` current: the device's copy of the
// scratch array, once per device.
hipError_t noalloc_init_device(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_status[device] = e;
    if (e == hipSuccess) g_ptr[device] = p;
    return e;
}

}  // namespace cds

extern "C" cds_status cds_sort_pairs_noalloc(cds_ctx* ctx, const uint64_t* keys_in, const uint32_t* values_in,
                                             int64_t count, int32_t end_bit, uint64_t* keys_out,
                                             uint32_t* values_out, uint32_t flags, void* stream_) {
    if (!ctx) return fail(CDS_ERR_INVALID_ARG, "context is NULL");
    if (flags & ~(CDS_OPT_SORT_ONESWEEP | CDS_OPT_SORT_REDUCE_SCAN) ||
        ((flags & CDS_OPT_SORT_ONESWEEP) && (flags & CDS_OPT_SORT_REDUCE_SCAN)))
        return fail(CDS_ERR_INVALID_ARG, "bad sort flags");
    if (count < 0 || end_bit < 1 || end_bit > 64) return fail(CDS_ERR_INVALID_ARG, "bad count or end_bit");
    if (count > kMaxPairs)
        return fail(CDS_ERR_CAPACITY, "cds_sort_pairs_noalloc sorts at most " + std::to_string(kMaxPairs) +
                                          " pairs (its scratch array is fixed)");
    if (count > 0 && (!keys_in || !values_in || !keys_out || !values_out))
        return fail(CDS_ERR_INVALID_ARG, "NULL array");
    if (count > 0 && ((const void*)keys_out == (const void*)keys_in ||
                      (const void*)values_out == (const void*)values_in))
        return fail(CDS_ERR_INVALID_ARG, "outputs may not alias inputs");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (count == 0) return CDS_OK;
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) base = static_cast<unsigned char*>(g_ptr[ctx->device]);
        if (!base)
            return hip_fail(ctx->device >= 0 && ctx->device < kMaxDevices ? g_status[ctx->device]
                                                                          : hipErrorInvalidDevice,
                            "scratch array address");
    }
    const SortAlgo algo = sort_algo_from_flags(flags);
    const int passes = (end_bit + 7) / 8;
    const int64_t parts = sort_partitions(count);
    if ((size_t)scan_block_sums_size(256 * parts) * sizeof(uint64_t) > kScanSumsBytes)
        return fail(CDS_ERR_CAPACITY, "scratch layout too small for the scan sums");
    SortWorkspace ws;
    ws.hist = reinterpret_cast<uint32_t*>(base + kOffHist);
    ws.status = reinterpret_cast<uint32_t*>(base + kOffStatus);
    ws.counters = reinterpret_cast<uint32_t*>(base + kOffCounters);
    ws.part_hist = reinterpret_cast<uint32_t*>(base + kOffPartHist);
    ws.bases = reinterpret_cast<uint32_t*>(base + kOffBases);
    ws.scan_sums = reinterpret_cast<uint64_t*>(base + kOffScanSums);
    ws.scan_total = reinterpret_cast<uint64_t*>(base + kOffScanTotal);
    ws.err = ctx->d_err;
    uint64_t* tmpk = reinterpret_cast<uint64_t*>(base + kOffKeys);
    uint32_t* tmpv = reinterpret_cast<uint32_t*>(base + kOffVals);
    // ping-pong so the last pass writes the caller's buffers and the input is never written
    uint64_t *ka, *kb;
    uint32_t *va, *vb;
    if (passes & 1) { ka = keys_out; va = values_out; kb = tmpk; vb = tmpv; }
    else            { ka = tmpk; va = tmpv; kb = keys_out; vb = values_out; }
    hipStream_t stream = (hipStream_t)stream_;
    // status words, partition counters and digit counts start at zero (fill kernels)
    if ((e = launch_sort_prepare(ws, count, passes, true, stream)) != hipSuccess) return hip_fail(e, "sort prepare");
    if (sort_uses_onesweep(count, algo) &&
        (e = launch_sort_histogram(keys_in, count, passes, 0, ws.hist, stream, end_bit)) != hipSuccess)
        return hip_fail(e, "sort histogram");
    if ((e = launch_sort_passes(keys_in, values_in, ka, va, kb, vb, count, passes, 0, ws, algo, stream, end_bit)) !=
        hipSuccess)
        return hip_fail(e, "sort passes");
    return CDS_OK;
}
