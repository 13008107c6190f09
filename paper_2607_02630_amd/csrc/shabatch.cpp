// shabatch.cpp -- sha256_batch: validation, ordering and staging of the
// message table, and the launch.
//
// Per (device, stream) the library keeps a ring of pinned staging slots of
// kMaxShaBatch records; a call orders its messages longest first (lanes of a
// wave then run for similar lengths), writes them to a free slot and launches
// the kernel on it: each lane reads its 32-byte record from the slot over
// PCIe (zero-copy), so there is no upload to order behind the previous launch
// and the host fills the next slot while the GPU hashes.  A slot is reused
// only after the event behind the launch that reads it fired.
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
    ShaRecord *staging[kShaSlots] = {};
    const ShaRecord *dev_view[kShaSlots] = {};   // the slots' device addresses
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
    for (int i = 0; i < kShaSlots; ++i) {
        // Coherent (fine-grained): the kernel reads the slot in place, and a
        // reused slot must never be served from a line cached by an earlier
        // launch.
        if (hipHostMalloc(reinterpret_cast<void **>(&c->staging[i]), bytes, hipHostMallocCoherent) != hipSuccess) {
            note_device_error(hipGetLastError());
            *rc = AES_ENOMEM;
            return nullptr;   // partially initialised context is leaked deliberately
        }
        void *view = nullptr;
        if (hipHostGetDevicePointer(&view, c->staging[i], 0) != hipSuccess || !view) {
            *rc = device_error();
            return nullptr;
        }
        c->dev_view[i] = static_cast<const ShaRecord *>(view);
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
        fill(c->staging[slot], first, m);
        // One lane per message; at most 16 workgroups of 256 lanes per CU,
        // extra messages looping in grid strides.
        const uint32_t groups = (m + 255) / 256;
        const int grid = static_cast<int>(std::min<uint32_t>(groups, static_cast<uint32_t>(16 * num_cus)));
        if ((rc = launch_sha256_batch(c->dev_view[slot], m, grid, st)) != AES_OK)
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
    thread_local std::vector<uint32_t> order;
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
    uint64_t lo = desc[0].len, hi = desc[0].len;
    for (size_t i = 0; i < n; ++i) {
        if (desc[i].reserved != 0)
            return AES_EINVAL;
        const int rc = check_sha(desc[i].in, desc[i].len, desc[i].digest);
        if (rc != AES_OK)
            return rc;
        lo = std::min<uint64_t>(lo, desc[i].len);
        hi = std::max<uint64_t>(hi, desc[i].len);
    }
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != AES_OK)
        return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto rec = [&](size_t i) {
        return ShaRecord{reinterpret_cast<uint64_t>(desc[i].in), desc[i].len,
                         reinterpret_cast<uint64_t>(desc[i].digest), 0};
    };
    if (lo == hi)   // equal lengths: the caller's order, written straight into staging
        return stage_and_launch(di.ordinal, st, n, di.num_cus, [&](ShaRecord *dst, size_t first, uint32_t m) {
            for (uint32_t i = 0; i < m; ++i)
                dst[i] = rec(first + i);
        });
    thread_local std::vector<uint32_t> order;
    length_order(n, [&](size_t i) { return desc[i].len; }, order);
    return stage_and_launch(di.ordinal, st, n, di.num_cus, [&](ShaRecord *dst, size_t first, uint32_t m) {
        for (uint32_t i = 0; i < m; ++i)
            dst[i] = rec(order[first + i]);
    });
}
