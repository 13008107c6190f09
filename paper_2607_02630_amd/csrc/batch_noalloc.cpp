// batch_noalloc.cpp -- aes_ctr_crypt_batch_noalloc: the batch launch with its
// descriptor table in a fixed device array of the library's own, for callers
// that must not allocate.
//
// aes_ctr_crypt_batch stages its table through per-stream contexts that the
// library allocates on first use (device table, pinned staging slots, graphs).
// This variant allocates nothing: the table lives in `scratch`, a file-scope
// device array that each GPU running the library holds until the process
// ends.  Its device address is taken with hipGetSymbolAddress once per device
// (on the first call on that device) and used for every copy and launch; the
// array's name itself is a host-side stand-in and is never handed to the
// runtime.  The table (header, descriptors, inline keys) is built on the
// calling thread's stack in pieces and copied into scratch with
// hipMemcpyAsync from that pageable memory (the runtime takes the bytes
// before the call returns), then the same persistent batch kernel runs on it.
// The header's tile counter is uploaded as 0 with every call, so nothing in
// scratch needs clearing.  All calls on one GPU share its scratch: calls that
// overlap on one GPU race.
#include <mutex>
#include <string.h>

#include "aesctr_internal.h"

namespace aesctr {
namespace {

// One launch of up to kMaxBatch requests, every key inline: 64 + 4096 * 64 +
// 4096 * 256 bytes = 1.25 MiB.
constexpr size_t kNoallocTableBytes = batch_table_bytes(kMaxBatch, kMaxBatch, 0);

static __device__ __align__(256) uint8_t scratch[kNoallocTableBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];

// Device address of this device's scratch (the current device's), set up on
// the first call on the device.
int scratch_ptr(int device, uint8_t **out)
{
    if (device < 0 || device >= kMaxDevices)
        return AES_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            note_device_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
            (void)hipGetLastError();
            return AES_EDEVICE;
        }
        g_scratch[device] = p;
    }
    *out = static_cast<uint8_t *>(g_scratch[device]);
    return AES_OK;
}

// Requests staged on the stack per copy: 64 * (64 + 256) = 20 KiB.
constexpr size_t kPiece = 64;

int copy_in(uint8_t *dst, const void *src, size_t bytes, hipStream_t st)
{
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
        note_device_error(hipGetLastError());
        return AES_EDEVICE;
    }
    return AES_OK;
}

}  // namespace
}  // namespace aesctr

using namespace aesctr;

extern "C" int aes_ctr_crypt_batch_noalloc(const aes_ctr_desc_t *desc, size_t n, void *stream)
{
    if (n == 0)
        return AES_OK;
    if (!desc)
        return AES_EINVAL;
    if (n > static_cast<size_t>(kMaxBatch))
        return AES_ETOOBIG;
    uint64_t total = 0;
    for (size_t i = 0; i < n; ++i) {
        const int rc = check_desc(desc[i]);
        if (rc != AES_OK)
            return rc;
        total += desc[i].len;
    }
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != AES_OK)
        return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        note_device_error(hipGetLastError());
        return AES_EDEVICE;
    }
    if (cs != hipStreamCaptureStatusNone)
        return AES_EINVAL;   // the copies read the caller's stack
    uint8_t *table;
    if ((rc = scratch_ptr(di.ordinal, &table)) != AES_OK)
        return rc;

    const uint32_t tile_blocks = static_cast<uint32_t>(batch_tile_bytes(total, di.num_cus) / 16);
    const int bpl = batch_blocks_per_lane();
    BatchHeader h{};
    h.n = static_cast<uint32_t>(n);
    h.tile_blocks = tile_blocks;
    h.next = 0;
    h.n_keys = static_cast<uint32_t>(n);
    h.n_install = 0;
    h.keys_off = static_cast<uint32_t>(batch_keys_off(n));
    h.install_off = static_cast<uint32_t>(batch_install_off(n, n));
    h.resident = 0;
    uint64_t tiles = 0;
    BatchDesc dpiece[kPiece];
    KeyRec kpiece[kPiece];
    for (size_t first = 0; first < n; first += kPiece) {
        const size_t m = n - first < kPiece ? n - first : kPiece;
        for (size_t i = 0; i < m; ++i) {
            make_batch_desc(desc[first + i], &dpiece[i], &kpiece[i]);
            dpiece[i].key = static_cast<uint32_t>(first + i);
            dpiece[i].tile0 = static_cast<uint32_t>(tiles);
            tiles += ((dpiece[i].len + 15) / 16 + tile_blocks - 1) / tile_blocks;
            if (tiles > 0x7fffffffu)
                return AES_ERANGE;
        }
        if ((rc = copy_in(table + sizeof(BatchHeader) + first * sizeof(BatchDesc), dpiece, m * sizeof(BatchDesc),
                          st)) != AES_OK ||
            (rc = copy_in(table + batch_keys_off(n) + first * sizeof(KeyRec), kpiece, m * sizeof(KeyRec), st)) !=
                AES_OK)
            return rc;
    }
    h.total_tiles = static_cast<uint32_t>(tiles);
    if ((rc = copy_in(table, &h, sizeof(h), st)) != AES_OK)
        return rc;
    const uint64_t grid = tiles < static_cast<uint64_t>(di.num_cus) ? (tiles ? tiles : 1) : di.num_cus;
    return launch_ctr_batch(table, static_cast<int>(grid), 1024, bpl, st);
}
