// shabatch.cpp -- sha256_batch: validation, ordering and staging of the
// message table, and the launch.
//
// Per (device, stream) the library keeps a device table of kMaxShaBatch
// records and a ring of pinned staging slots; a call orders its messages
// longest first (lanes of a wave then run for similar lengths), writes them
// to a free slot, copies the slot to the table and launches the kernel.  A
// slot is reused only after the event behind its last launch fired; launches
// on one stream are ordered, so the single device table is never
// overwritten while a kernel reads it.
#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <string.h>
#include <vector>

#include "../../include/shabatch.h"
#include "shabatch_internal.h"

namespace aesctr {
namespace {

constexpr int kShaSlots = 2;

struct ShaCtx {
    std::mutex mu;
    ShaRecord *dev = nullptr;
    ShaRecord *staging[kShaSlots] = {};
    hipEvent_t done[kShaSlots] = {};
    bool used[kShaSlots] = {};
    int next = 0;
};

std::mutex g_sha_mu;
// Contexts live until process exit (see batch.cpp for why).
std::map<std::pair<int, void *>, ShaCtx *> g_sha;

ShaCtx *get_ctx(int device, void *stream, int *rc)
{
    std::lock_guard<std::mutex> lk(g_sha_mu);
    auto it = g_sha.find({device, stream});
    if (it != g_sha.end()) {
        *rc = AES_OK;
        return it->second;
    }
    ShaCtx *c = new ShaCtx();
    const size_t bytes = sizeof(ShaRecord) * kMaxShaBatch;
    if (hipMalloc(reinterpret_cast<void **>(&c->dev), bytes) != hipSuccess) {
        note_device_error(hipGetLastError());
        *rc = AES_ENOMEM;
        return nullptr;   // partially initialised context is leaked deliberately
    }
    for (int i = 0; i < kShaSlots; ++i) {
        if (hipHostMalloc(reinterpret_cast<void **>(&c->staging[i]), bytes, hipHostMallocDefault) != hipSuccess) {
            note_device_error(hipGetLastError());
            *rc = AES_ENOMEM;
            return nullptr;
        }
        if (hipEventCreateWithFlags(&c->done[i], hipEventDisableTiming) != hipSuccess) {
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

int launch_sha_records(int device, hipStream_t st, const ShaRecord *recs, size_t n, int num_cus)
{
    if (n == 0)
        return AES_OK;
    int rc;
    ShaCtx *c = get_ctx(device, st, &rc);
    if (!c)
        return rc;

    // Longest first, so lanes of a wave (consecutive records) hash similar
    // lengths: a stable counting sort on the bit length of len (O(n); equal
    // lengths keep the caller's order and skip the pass).
    thread_local std::vector<uint32_t> order;
    order.resize(n);
    uint64_t lo = recs[0].len, hi = recs[0].len;
    for (size_t i = 1; i < n; ++i) {
        lo = std::min<uint64_t>(lo, recs[i].len);
        hi = std::max<uint64_t>(hi, recs[i].len);
    }
    if (lo == hi) {
        std::iota(order.begin(), order.end(), 0u);
    } else {
        auto bucket = [](uint64_t len) { return 64 - __builtin_clzll(len | 1); };   // 1..62
        size_t start[66] = {};
        for (size_t i = 0; i < n; ++i)
            ++start[65 - bucket(recs[i].len)];
        size_t acc = 0;
        for (size_t &v : start) {
            const size_t cnt = v;
            v = acc;
            acc += cnt;
        }
        for (size_t i = 0; i < n; ++i)
            order[start[65 - bucket(recs[i].len)]++] = static_cast<uint32_t>(i);
    }

    std::lock_guard<std::mutex> lk(c->mu);
    for (size_t first = 0; first < n; first += kMaxShaBatch) {
        const uint32_t m = static_cast<uint32_t>(std::min<size_t>(n - first, kMaxShaBatch));
        const int slot = c->next;
        c->next = (c->next + 1) % kShaSlots;
        if (c->used[slot] && hipEventSynchronize(c->done[slot]) != hipSuccess)
            return device_error();
        ShaRecord *s = c->staging[slot];
        for (uint32_t i = 0; i < m; ++i)
            s[i] = recs[order[first + i]];
        if (hipMemcpyAsync(c->dev, s, sizeof(ShaRecord) * m, hipMemcpyHostToDevice, st) != hipSuccess)
            return device_error();
        // One lane per message; at most 16 workgroups of 256 lanes per CU,
        // extra messages looping in grid strides.
        const uint32_t groups = (m + 255) / 256;
        const int grid = static_cast<int>(std::min<uint32_t>(groups, static_cast<uint32_t>(16 * num_cus)));
        if ((rc = launch_sha256_batch(c->dev, m, grid, st)) != AES_OK)
            return rc;
        if (hipEventRecord(c->done[slot], st) != hipSuccess)
            return device_error();
        c->used[slot] = true;
    }
    return AES_OK;
}

}  // namespace aesctr

using namespace aesctr;

extern "C" int sha256_batch(const sha256_desc_t *desc, size_t n, void *stream)
{
    if (n == 0)
        return AES_OK;
    if (!desc)
        return AES_EINVAL;
    for (size_t i = 0; i < n; ++i) {
        if (desc[i].reserved != 0)
            return AES_EINVAL;
        const int rc = check_sha(desc[i].in, desc[i].len, desc[i].digest);
        if (rc != AES_OK)
            return rc;
    }
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != AES_OK)
        return rc;
    thread_local std::vector<ShaRecord> recs;
    recs.resize(n);
    for (size_t i = 0; i < n; ++i)
        recs[i] = ShaRecord{reinterpret_cast<uint64_t>(desc[i].in), desc[i].len,
                            reinterpret_cast<uint64_t>(desc[i].digest), 0};
    return launch_sha_records(di.ordinal, static_cast<hipStream_t>(stream), recs.data(), n, di.num_cus);
}
