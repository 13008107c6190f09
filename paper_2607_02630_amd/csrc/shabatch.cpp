// shabatch.cpp -- sha256_batch: validation, ordering and staging of the
// message table, and the launch.
//
// Per (device, stream) the library keeps two staging slots of kMaxShaBatch
// records, each a pinned host buffer with a device copy.  A call orders its
// messages longest first (lanes of a wave then run for similar lengths) and
// cuts them into launches of up to kMaxShaBatch records:
//  * a launch queued on an idle stream (the first of a call, when nothing
//    else is queued) reads its records from the pinned slot in place, over
//    PCIe (zero-copy), so nothing is uploaded ahead of it;
//  * every other launch's records are uploaded to the slot's device copy on
//    a side stream while the work queued before it runs, and the launch
//    waits for that upload only.
// A slot is refilled only after the event behind the launch that read it
// fired, and the host fills the next slot while the GPU hashes.
#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <string.h>
#include <vector>

#include "../../include/shabatch.h"
#include "host_pool.h"
#include "shabatch_internal.h"

namespace aesctr {
namespace {

constexpr int kShaSlots = 2;
// Descriptors per part of the host's parallel validation and staging.
constexpr size_t kShaGrain = 16384;

struct ShaCtx {
    std::mutex mu;
    ShaRecord *staging[kShaSlots] = {};
    const ShaRecord *host_view[kShaSlots] = {};  // the pinned slots' device addresses
    ShaRecord *dev_copy[kShaSlots] = {};         // device-memory copies of the slots
    hipEvent_t done[kShaSlots] = {};             // the launch that read the slot
    hipEvent_t uploaded[kShaSlots] = {};         // the slot's upload to dev_copy
    hipStream_t upload = nullptr;                // side stream of the uploads
    bool used[kShaSlots] = {};
    int next = 0;
};

std::mutex g_sha_mu;
// Contexts live until process exit (see batch.cpp for why); a retired
// stream's context goes to its device's free list for the next stream
// (release_sha_stream).  The coherent slots in particular are never freed.
std::map<std::pair<int, void *>, ShaCtx *> g_sha;
std::map<int, std::vector<ShaCtx *>> g_sha_free;

ShaCtx *get_ctx(int device, void *stream, int *rc)
{
    std::lock_guard<std::mutex> lk(g_sha_mu);
    auto it = g_sha.find({device, stream});
    if (it != g_sha.end()) {
        *rc = AES_OK;
        return it->second;
    }
    std::vector<ShaCtx *> &fl = g_sha_free[device];
    if (!fl.empty()) {
        ShaCtx *c = fl.back();
        fl.pop_back();
        g_sha[{device, stream}] = c;
        *rc = AES_OK;
        return c;
    }
    ShaCtx *c = new ShaCtx();
    const size_t bytes = sizeof(ShaRecord) * kMaxShaBatch;
    // A partially initialised context is leaked deliberately on error.
    if (hipStreamCreateWithFlags(&c->upload, hipStreamNonBlocking) != hipSuccess) {
        *rc = device_error();
        return nullptr;
    }
    for (int i = 0; i < kShaSlots; ++i) {
        // Coherent (fine-grained): the kernel reads the slot in place, and a
        // reused slot must never be served from a line cached by an earlier
        // launch.
        if (hipHostMalloc(reinterpret_cast<void **>(&c->staging[i]), bytes, hipHostMallocCoherent) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&c->dev_copy[i]), bytes) != hipSuccess) {
            note_device_error(hipGetLastError());
            *rc = AES_ENOMEM;
            return nullptr;
        }
        void *view = nullptr;
        if (hipHostGetDevicePointer(&view, c->staging[i], 0) != hipSuccess || !view) {
            *rc = device_error();
            return nullptr;
        }
        c->host_view[i] = static_cast<const ShaRecord *>(view);
        if (hipEventCreateWithFlags(&c->done[i], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->uploaded[i], hipEventDisableTiming) != hipSuccess) {
            *rc = device_error();
            return nullptr;
        }
    }
    g_sha[{device, stream}] = c;
    *rc = AES_OK;
    return c;
}

}  // namespace
}  // namespace aesctr

namespace aesctr {

void release_sha_stream(int device, hipStream_t st)
{
    ShaCtx *c = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_sha_mu);
        auto it = g_sha.find({device, static_cast<void *>(st)});
        if (it == g_sha.end())
            return;
        c = it->second;
        g_sha.erase(it);
    }
    {
        std::lock_guard<std::mutex> lk(c->mu);
        for (int i = 0; i < kShaSlots; ++i) {
            if (c->used[i] && hipEventSynchronize(c->done[i]) != hipSuccess)
                note_device_error(hipGetLastError());
            c->used[i] = false;
        }
        c->next = 0;
    }
    std::lock_guard<std::mutex> lk(g_sha_mu);
    g_sha_free[device].push_back(c);
}

int check_sha(const void *in, uint64_t len, const void *digest)
{
    if (!digest)
        return AES_EINVAL;
    if (len == 0)
        return AES_OK;
    if (!in)
        return AES_EINVAL;
    if (len > (uint64_t(1) << 61) - 1)
        return AES_ERANGE;
    const uintptr_t a = reinterpret_cast<uintptr_t>(in);
    const uintptr_t b = reinterpret_cast<uintptr_t>(digest);
    if (a > UINTPTR_MAX - len || b > UINTPTR_MAX - 32)
        return AES_EINVAL;
    if (a < b + 32 && b < a + len)
        return AES_EOVERLAP;
    return AES_OK;
}

namespace {

// Stages n records, produced by fill(dst, first, m) for records
// [first, first + m) in launch order, and launches them (kMaxShaBatch each).
template <class Fill>
int stage_and_launch(int device, hipStream_t st, size_t n, int num_cus, Fill fill)
{
    int rc;
    ShaCtx *c = get_ctx(device, st, &rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    for (size_t first = 0; first < n; first += kMaxShaBatch) {
        const uint32_t m = static_cast<uint32_t>(std::min<size_t>(n - first, kMaxShaBatch));
        const int slot = c->next;
        c->next = (c->next + 1) % kShaSlots;
        if (c->used[slot] && hipEventSynchronize(c->done[slot]) != hipSuccess)
            return device_error();
        ShaRecord *dst = c->staging[slot];
        HostPool::get().parallel_for(m, kShaGrain, [&](size_t, size_t b, size_t e) {
            fill(dst + b, first + b, static_cast<uint32_t>(e - b));
        });
        // One lane per message; at most 16 workgroups of 256 lanes per CU,
        // extra messages looping in grid strides.
        const uint32_t groups = (m + 255) / 256;
        const int grid = static_cast<int>(std::min<uint32_t>(groups, static_cast<uint32_t>(16 * num_cus)));
        const ShaRecord *recs = c->host_view[slot];
        if (first > 0 || hipStreamQuery(st) != hipSuccess) {
            // The upload may start at once: it waits for nothing on `st`
            // (the slot's previous reader finished, see above), so it runs
            // beside the work queued before the launch.
            recs = c->dev_copy[slot];
            if (hipMemcpyAsync(c->dev_copy[slot], c->staging[slot], sizeof(ShaRecord) * m, hipMemcpyHostToDevice,
                               c->upload) != hipSuccess ||
                hipEventRecord(c->uploaded[slot], c->upload) != hipSuccess ||
                hipStreamWaitEvent(st, c->uploaded[slot], 0) != hipSuccess)
                return device_error();
        }
        if ((rc = launch_sha256_batch(recs, m, grid, st)) != AES_OK)
            return rc;
        if (hipEventRecord(c->done[slot], st) != hipSuccess)
            return device_error();
        c->used[slot] = true;
    }
    return AES_OK;
}

// Launch order: longest first, so lanes of a wave (consecutive records) hash
// similar lengths -- a stable counting sort on the bit length (O(n)).
template <class LenOf>
void length_order(size_t n, LenOf len_of, std::vector<uint32_t> &order)
{
    auto bucket = [](uint64_t len) { return 64 - __builtin_clzll(len | 1); };   // 1..62
    size_t start[66] = {};
    for (size_t i = 0; i < n; ++i)
        ++start[65 - bucket(len_of(i))];
    size_t acc = 0;
    for (size_t &v : start) {
        const size_t cnt = v;
        v = acc;
        acc += cnt;
    }
    order.resize(n);
    for (size_t i = 0; i < n; ++i)
        order[start[65 - bucket(len_of(i))]++] = static_cast<uint32_t>(i);
}

}  // namespace

int launch_sha_records(int device, hipStream_t st, const ShaRecord *recs, size_t n, int num_cus)
{
    if (n == 0)
        return AES_OK;
    // The fill runs on pool threads too: they must see this thread's order
    // (a lambda does not capture a thread_local, it names the running
    // thread's own), hence the plain reference.
    thread_local std::vector<uint32_t> tl_order;
    std::vector<uint32_t> &order = tl_order;
    length_order(n, [&](size_t i) { return recs[i].len; }, order);
    return stage_and_launch(device, st, n, num_cus, [&](ShaRecord *dst, size_t first, uint32_t m) {
        for (uint32_t i = 0; i < m; ++i)
            dst[i] = recs[order[first + i]];
    });
}

}  // namespace aesctr

using namespace aesctr;

extern "C" int sha256_batch(const sha256_desc_t *desc, size_t n, void *stream)
{
    if (n == 0)
        return AES_OK;
    if (!desc)
        return AES_EINVAL;
    // Validation and the length range, over parts in parallel; the status of
    // the first failing descriptor wins, as in a serial scan.
    struct Scan {
        int rc;
        uint64_t lo, hi;
    };
    HostPool &pool = HostPool::get();
    const size_t parts = HostPool::parts(n, kShaGrain);
    Scan scan[HostPool::kMaxParts];
    pool.parallel_for(n, kShaGrain, [&](size_t p, size_t b, size_t e) {
        Scan r{AES_OK, UINT64_MAX, 0};
        for (size_t i = b; i < e && r.rc == AES_OK; ++i) {
            r.rc = desc[i].reserved != 0 ? AES_EINVAL : check_sha(desc[i].in, desc[i].len, desc[i].digest);
            r.lo = std::min<uint64_t>(r.lo, desc[i].len);
            r.hi = std::max<uint64_t>(r.hi, desc[i].len);
        }
        scan[p] = r;
    });
    uint64_t lo = UINT64_MAX, hi = 0;
    for (size_t p = 0; p < parts; ++p) {
        if (scan[p].rc != AES_OK)
            return scan[p].rc;
        lo = std::min(lo, scan[p].lo);
        hi = std::max(hi, scan[p].hi);
    }
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != AES_OK)
        return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // The call cannot be captured into a caller's graph: the graph would
    // keep reading staging slots that later calls rewrite.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess)
        return device_error();
    if (cs != hipStreamCaptureStatusNone)
        return AES_EINVAL;
    auto rec = [&](size_t i) {
        return ShaRecord{reinterpret_cast<uint64_t>(desc[i].in), desc[i].len,
                         reinterpret_cast<uint64_t>(desc[i].digest), 0};
    };
    if (lo == hi)   // equal lengths: the caller's order, written straight into staging
        return stage_and_launch(di.ordinal, st, n, di.num_cus, [&](ShaRecord *dst, size_t first, uint32_t m) {
            for (uint32_t i = 0; i < m; ++i)
                dst[i] = rec(first + i);
        });
    thread_local std::vector<uint32_t> tl_order;
    std::vector<uint32_t> &order = tl_order;   // see launch_sha_records
    length_order(n, [&](size_t i) { return desc[i].len; }, order);
    return stage_and_launch(di.ordinal, st, n, di.num_cus, [&](ShaRecord *dst, size_t first, uint32_t m) {
        for (uint32_t i = 0; i < m; ++i)
            dst[i] = rec(order[first + i]);
    });
}
