// engine.cpp -- the serving engine: submit / poll / wait over continuous
// batching on HIP streams.
//
// One driver thread per engine owns the device side.  In a loop it
//   1. polls the event behind each stream's in-flight launch (the paper's
//      completion test by event query, Sec. 6 setup) and retires finished
//      launches, releasing their bytes from the budget;
//   2. for every stream with nothing in flight, takes everything admitted so
//      far (FIFO, within the byte budget and per-launch limits) and launches
//      it as one persistent batch kernel -- requests that arrived while other
//      launches were running join the next one, and launches on different
//      streams overlap on the device;
//   3. sleeps when there is nothing queued and nothing in flight, after
//      polling for new work for kIdleSpinNs (a sleeping driver costs the
//      next request a thread wake-up on its way to the GPU).
// Request records (pointers, counter parameters, expanded key material) are
// built on the submitting thread, so the driver only copies them into the
// launch's descriptor table.
//
// With host_buffers the request buffers are pinned host memory (hipHostMalloc)
// that the kernel reads and writes directly over PCIe; otherwise they are
// device memory.
#include <algorithm>
#include <atomic>
#include <errno.h>
#include <sys/eventfd.h>
#include <thread>
#include <unistd.h>
#include <vector>

#include "aesctr_internal.h"
#include "engine_core.h"
#include "key_cache.h"
#include "shabatch_internal.h"

using aesctr::BatchDesc;
using aesctr::KeyCache;
using aesctr::RequestRec;
using Core = aesctr::EngineCore<RequestRec>;
using Req = Core::Req;
using aesctr::note_device_error;

struct aes_engine {
    aes_engine(uint64_t budget, size_t max_reqs, uint64_t max_bytes, int key_slots)
        : core(budget, max_reqs, max_bytes), keys(key_slots),
          inline_of_slot(static_cast<size_t>(key_slots), -1), inline_epoch(static_cast<size_t>(key_slots), 0)
    {
    }

    Core core;
    int device = 0;
    int num_cus = 0;
    int host_buffers = 0;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<std::vector<Req>> inflight;
    std::vector<int> inflight_status;   // status the in-flight batch completes with
    std::vector<std::vector<KeyCache::Ref>> inflight_keys;   // key-slot references of each stream's launch
    std::thread driver;
    int efd = -1;

    // Resident key schedules (key_slots > 0): the device table of key records
    // and, on the driver thread, the cache that assigns its slots.
    KeyCache keys;
    void *key_table = nullptr;
    std::atomic<uint64_t> key_hits{0}, key_misses{0};
    uint64_t key_hits_base = 0, key_misses_base = 0;
    // Inline copy of a key this launch installs, per slot (valid when the
    // slot's epoch is the launch's), so requests sharing a new key carry it once.
    std::vector<int32_t> inline_of_slot;
    std::vector<uint32_t> inline_epoch;
    uint32_t epoch = 0;
    // Staging of the launch being formed (driver thread).
    std::vector<BatchDesc> descs;
    std::vector<aesctr::KeyRec> keyrecs;
    std::vector<aesctr::InstallRec> installs;
};

namespace {

constexpr int kMaxStreams = 16;
constexpr int kMaxKeySlots = 1 << 16;   // 16 MiB of resident key records

void notify_fd(int fd)
{
    if (fd >= 0) {
        uint64_t one = 1;
        ssize_t r = write(fd, &one, sizeof(one));
        (void)r;   // EAGAIN only when the counter is saturated: still readable
    }
}

// Tile size of a zero-copy batch (host_buffers): about 256 tiles, 2-64 KiB,
// a multiple of 2 KiB.  The payload crosses PCIe, which a few hundred KiB in
// flight keep busy, so 256 waves suffice; each then runs several 2 KiB steps,
// and one wave's writes overlap another's reads.  With one step per wave (the
// device-memory sizing) a whole batch is read before any of it is written
// back, and a lone 8 MiB request ran at 30 GB/s of payload.
uint64_t zero_copy_tile_bytes(uint64_t batch_bytes)
{
    const uint64_t tile = (batch_bytes / 256 + 2047) & ~uint64_t(2047);
    return tile < 2048 ? 2048 : tile > 65536 ? 65536 : tile;
}

// Waits for everything queued on stream s, after a launch call failed
// part-way (a call that launches several chunks may fail after the first):
// the batch is then completed at once, and no kernel may still touch its
// buffers.
int drain_after_error(aes_engine *e, int s, int rc)
{
    (void)hipStreamSynchronize(e->streams[s]);
    return rc;
}

// Where a launch reads request q's round keys: a resident slot, or an inline
// copy in the launch's table (installed into a slot when one is free).
// Records the slot reference for release at completion.
uint32_t place_key(aes_engine *e, const RequestRec &q, std::vector<KeyCache::Ref> &refs)
{
    const KeyCache::Ref r = e->keys.acquire(q.key.rk, q.d.nr);
    if (r.slot >= 0)
        refs.push_back(r);
    if (r.resident) {
        e->key_hits.fetch_add(1, std::memory_order_relaxed);
        return aesctr::kKeyResident | static_cast<uint32_t>(r.slot);
    }
    if (e->keys.slots() > 0)
        e->key_misses.fetch_add(1, std::memory_order_relaxed);
    if (r.pending >= 0 && e->inline_epoch[r.pending] == e->epoch)
        return static_cast<uint32_t>(e->inline_of_slot[r.pending]);
    const uint32_t idx = static_cast<uint32_t>(e->keyrecs.size());
    e->keyrecs.push_back(q.key);
    if (r.install) {
        e->installs.push_back(aesctr::InstallRec{idx, static_cast<uint32_t>(r.slot)});
        e->inline_of_slot[r.slot] = static_cast<int32_t>(idx);
        e->inline_epoch[r.slot] = e->epoch;
    }
    return idx;
}

void release_keys(aes_engine *e, int s, bool ok)
{
    for (const KeyCache::Ref &r : e->inflight_keys[s])
        e->keys.release(r, ok);
    e->inflight_keys[s].clear();
}

// Launches one batch on stream s and records the stream's completion event.
// Returns the batch's status.  *launched tells whether any work reached the
// stream: if so the caller must keep the batch in flight until the event
// fires, even when the status is an error, so no buffer is released while a
// kernel may still touch it.  The batch's key-slot references are left in
// e->inflight_keys[s] either way.
int launch_batch(aes_engine *e, int s, const std::vector<Req> &batch, std::vector<aesctr::ShaRecord> &hashes,
                 bool *launched)
{
    *launched = false;
    // Cipher records go to the batch kernel, hash records (nr == 0) to the
    // hash kernel; both run on this stream before its completion event.
    e->descs.clear();
    e->keyrecs.clear();
    e->installs.clear();
    hashes.clear();
    if (++e->epoch == 0) {
        std::fill(e->inline_epoch.begin(), e->inline_epoch.end(), 0);
        e->epoch = 1;
    }
    uint64_t bytes = 0;
    for (const Req &q : batch) {
        if (q.rec.d.nr == 0) {
            hashes.push_back(aesctr::ShaRecord{q.rec.d.in, q.rec.d.len, q.rec.d.out, 0});
        } else {
            BatchDesc d = q.rec.d;
            d.key = place_key(e, q.rec, e->inflight_keys[s]);
            e->descs.push_back(d);
            bytes += d.len;
        }
    }
    int rc = AES_OK;
    if (!e->descs.empty()) {
        // Tile size sized to the batch (see batch_tile_bytes); one workgroup
        // per CU at most, and no more workgroups than tiles, so a batch of a
        // few requests spreads over many CUs and leaves the rest to the other
        // stream.
        const uint64_t cus = static_cast<uint64_t>(e->num_cus);
        const uint64_t tile = e->host_buffers ? zero_copy_tile_bytes(bytes) : aesctr::batch_tile_bytes(bytes, e->num_cus);
        uint64_t tiles = 0;
        const uint64_t tile_blocks = tile / 16;
        for (const BatchDesc &r : e->descs)
            tiles += ((r.len + 15) / 16 + tile_blocks - 1) / tile_blocks;
        uint64_t grid = tiles < cus ? tiles : cus;
        if (grid < 1)
            grid = 1;
        aesctr::LaunchSpec spec;
        spec.descs = e->descs.data();
        spec.n = e->descs.size();
        spec.keys = e->keyrecs.data();
        spec.n_keys = e->keyrecs.size();
        spec.installs = e->installs.data();
        spec.n_install = e->installs.size();
        spec.resident = reinterpret_cast<uint64_t>(e->key_table);
        // Small batches go in the kernel arguments (no upload ahead of the
        // launch) except for zero-copy buffers: there the upload's delay
        // lets more requests join each launch, and launches of a few
        // requests kept too little PCIe traffic in flight (at 90% of
        // saturation the p99 rose from 2.5 to 4.3 ms).
        rc = aesctr::launch_spec(e->device, e->streams[s], spec, static_cast<int>(tile), static_cast<int>(grid),
                                 aesctr::batch_blocks_per_lane(), false, e->host_buffers == 0);
        if (rc != AES_OK)
            return drain_after_error(e, s, rc);
        *launched = true;
    }
    if (!hashes.empty()) {
        const int hrc =
            aesctr::launch_sha_records(e->device, e->streams[s], hashes.data(), hashes.size(), e->num_cus);
        if (hrc != AES_OK && !*launched)
            return drain_after_error(e, s, hrc);
        rc = hrc;
        *launched = true;
    }
    if (hipEventRecord(e->events[s], e->streams[s]) != hipSuccess) {
        note_device_error(hipGetLastError());
        // No event to poll: wait for whatever reached the stream here.
        (void)hipStreamSynchronize(e->streams[s]);
        *launched = false;
        return AES_EDEVICE;
    }
    return rc;
}

// How long an idle driver keeps polling for work before it sleeps.
constexpr int64_t kIdleSpinNs = 100000;

void drive(aes_engine *e)
{
    if (hipSetDevice(e->device) != hipSuccess) {
        note_device_error(hipGetLastError());
        e->core.close();
        e->core.cancel_queued(AES_EDEVICE);
        return;
    }
    const int ns = static_cast<int>(e->streams.size());
    std::vector<Req> batch;
    std::vector<aesctr::ShaRecord> hashes;
    int active = 0;
    int64_t busy_since = 0;
    int64_t idle_since = -1;
    for (;;) {
        bool progressed = false;
        for (int s = 0; s < ns; ++s) {
            if (e->inflight[s].empty())
                continue;
            hipError_t q = hipEventQuery(e->events[s]);
            if (q == hipErrorNotReady)
                continue;
            const int status = q == hipSuccess ? e->inflight_status[s] : AES_EDEVICE;
            if (q != hipSuccess)
                note_device_error(hipGetLastError());
            const int64_t now = Core::now_ns();
            release_keys(e, s, q == hipSuccess);
            e->core.complete(e->inflight[s], status, now);
            e->inflight[s].clear();
            if (--active == 0)
                e->core.add_busy(now - busy_since);
            progressed = true;
        }
        for (int s = 0; s < ns; ++s) {
            if (!e->inflight[s].empty())
                continue;
            if (!e->core.take_batch(batch))
                break;
            bool launched = false;
            const int rc = launch_batch(e, s, batch, hashes, &launched);
            if (!launched) {
                release_keys(e, s, false);
                e->core.complete(batch, rc, Core::now_ns());
                continue;
            }
            e->inflight_status[s] = rc;
            if (active++ == 0)
                busy_since = Core::now_ns();
            e->inflight[s].swap(batch);
            progressed = true;
        }
        if (progressed) {
            idle_since = -1;
        } else if (active > 0) {
            std::this_thread::yield();
        } else {
            if (e->core.closing_and_drained())
                break;
            const int64_t now = Core::now_ns();
            if (idle_since < 0)
                idle_since = now;
            if (now - idle_since < kIdleSpinNs) {
                std::this_thread::yield();
            } else {
                idle_since = -1;
                e->core.wait_for_work(2000000);
            }
        }
    }
}

}  // namespace

extern "C" int aes_engine_create(const aes_engine_cfg_t *cfg, aes_engine_t **out)
{
    if (!out)
        return AES_EINVAL;
    *out = nullptr;
    aes_engine_cfg_t c{};
    if (cfg)
        c = *cfg;
    const uint64_t budget = c.budget_bytes ? c.budget_bytes : (4ull << 30);
    const int nstreams = c.n_streams ? c.n_streams : 2;
    const int max_reqs = c.max_batch_reqs > 0 && c.max_batch_reqs < aesctr::kMaxBatch ? c.max_batch_reqs
                                                                                        : aesctr::kMaxBatch;
    // Default per-launch cap: 256 MiB (or the budget).  Measured on the
    // serving mix: 6% below the uncapped saturation rate, with the p99 at 90%
    // of saturation 26% lower; a request larger than the cap runs alone.
    const uint64_t max_bytes = c.max_batch_bytes ? c.max_batch_bytes : std::min<uint64_t>(budget, 256ull << 20);
    if (nstreams < 1 || nstreams > kMaxStreams || c.max_batch_reqs < 0 || c.key_slots < 0 ||
        c.key_slots > kMaxKeySlots || (c.host_buffers != 0 && c.host_buffers != 1))
        return AES_EINVAL;

    int dev = c.device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
        note_device_error(hipGetLastError());
        return AES_EDEVICE;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || dev >= ndev) {
        note_device_error(hipGetLastError());
        return AES_EDEVICE;
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(dev) != hipSuccess) {
        note_device_error(hipGetLastError());
        return AES_EDEVICE;
    }
    aesctr::DeviceInfo di;
    int rc = aesctr::device_info(&di);
    if (rc != AES_OK) {
        if (prev >= 0)
            (void)hipSetDevice(prev);
        return rc;
    }

    aes_engine *e = new aes_engine(budget, static_cast<size_t>(max_reqs), max_bytes, c.key_slots);
    e->device = dev;
    e->num_cus = di.num_cus;
    e->host_buffers = c.host_buffers;
    e->inflight.resize(nstreams);
    e->inflight_keys.resize(nstreams);
    e->inflight_status.assign(nstreams, AES_OK);
    if (c.key_slots > 0 && hipMalloc(&e->key_table, static_cast<size_t>(c.key_slots) * sizeof(aesctr::KeyRec)) !=
                               hipSuccess) {
        e->key_table = nullptr;
        rc = AES_ENOMEM;
    }
    for (int s = 0; s < nstreams && rc == AES_OK; ++s) {
        hipStream_t st;
        hipEvent_t ev;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            rc = AES_EDEVICE;
            break;
        }
        e->streams.push_back(st);
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            rc = AES_EDEVICE;
            break;
        }
        e->events.push_back(ev);
    }
    if (prev >= 0)
        (void)hipSetDevice(prev);
    if (rc != AES_OK) {
        note_device_error(hipGetLastError());
        for (hipStream_t st : e->streams)
            (void)hipStreamDestroy(st);
        for (hipEvent_t ev : e->events)
            (void)hipEventDestroy(ev);
        if (e->key_table)
            (void)hipFree(e->key_table);
        delete e;
        return rc;
    }
    e->efd = eventfd(0, EFD_NONBLOCK | EFD_CLOEXEC);
    const int fd = e->efd;
    e->core.set_on_complete([fd] { notify_fd(fd); });
    e->driver = std::thread(drive, e);
    *out = e;
    return AES_OK;
}

extern "C" int aes_engine_destroy(aes_engine_t *e)
{
    if (!e)
        return AES_EINVAL;
    e->core.close();
    if (e->driver.joinable())
        e->driver.join();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(e->device);
    // The driver has retired every launch; the streams' staging contexts go
    // back to the device's pools for the next engine.
    for (hipStream_t st : e->streams) {
        aesctr::release_batch_stream(e->device, st);
        aesctr::release_sha_stream(e->device, st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t ev : e->events)
        (void)hipEventDestroy(ev);
    if (e->key_table)
        (void)hipFree(e->key_table);
    if (prev >= 0)
        (void)hipSetDevice(prev);
    if (e->efd >= 0)
        close(e->efd);
    delete e;
    return AES_OK;
}

namespace {

// Device address of pinned host memory; AES_EINVAL if p is not memory the
// device can reach (e.g. pageable host memory).
int host_to_device(const void *p, uint64_t *dev)
{
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        note_device_error(hipGetLastError());
        return AES_EINVAL;
    }
    if (at.type != hipMemoryTypeHost || !at.devicePointer)
        return AES_EINVAL;
    *dev = reinterpret_cast<uint64_t>(at.devicePointer);
    return AES_OK;
}

}  // namespace

extern "C" int aes_submit_at(aes_engine_t *e, const aes_ctr_desc_t *d, int64_t t_arrival_ns, uint64_t *ticket)
{
    if (!e || !d || !ticket || t_arrival_ns < 0)
        return AES_EINVAL;
    int rc;
    Req r;
    if (d->flags == AES_FLAG_SHA256) {
        // A hash request: in = message, out = 32-byte digest.  Its record
        // carries nr = 0, which no cipher record has.
        if (d->reserved != 0)
            return AES_EINVAL;
        if ((rc = aesctr::check_sha(d->in, d->len, d->out)) != AES_OK)
            return rc;
        r.rec.d = BatchDesc{};
        r.rec.d.in = reinterpret_cast<uint64_t>(d->in);
        r.rec.d.out = reinterpret_cast<uint64_t>(d->out);
        r.rec.d.len = d->len;
        r.rec.d.nr = 0;
        if (e->host_buffers) {
            uint64_t din = 0, dout = 0;
            if ((d->len > 0 && (rc = host_to_device(d->in, &din)) != AES_OK) ||
                (rc = host_to_device(d->out, &dout)) != AES_OK)
                return rc;
            r.rec.d.in = din;
            r.rec.d.out = dout;
        }
        r.bytes = d->len + 32 + sizeof(aesctr::ShaRecord);
        r.payload = d->len;
        return e->core.submit(std::move(r), ticket, t_arrival_ns);
    }
    if ((rc = aesctr::check_desc(*d)) != AES_OK)
        return rc;
    // Admission weight: the request's buffers while it is in flight (input
    // and output, once when in place) and its staged records (descriptor and,
    // unless its key is resident, an inline key record).
    r.bytes = (d->in == d->out ? 1 : 2) * d->len + aes_engine_request_overhead();
    r.payload = d->len;
    aesctr::make_batch_record(*d, &r.rec);
    if (e->host_buffers && d->len > 0) {
        // The kernel reads and writes the pinned host buffers directly.
        uint64_t din = 0, dout = 0;
        if ((rc = host_to_device(d->in, &din)) != AES_OK || (rc = host_to_device(d->out, &dout)) != AES_OK)
            return rc;
        r.rec.d.in = din;
        r.rec.d.out = dout;
        r.rec.d.aligned = ((din | dout) & 15) == 0;
    }
    return e->core.submit(std::move(r), ticket, t_arrival_ns);
}

extern "C" int aes_submit(aes_engine_t *e, const aes_ctr_desc_t *d, uint64_t *ticket)
{
    return aes_submit_at(e, d, e ? Core::now_ns() : 0, ticket);
}

extern "C" int aes_poll(aes_engine_t *e, uint64_t ticket)
{
    if (!e)
        return AES_EINVAL;
    return e->core.poll(ticket);
}

extern "C" int aes_wait(aes_engine_t *e, uint64_t ticket, int64_t timeout_us)
{
    if (!e)
        return AES_EINVAL;
    return e->core.wait(ticket, timeout_us);
}

extern "C" int aes_engine_stats(aes_engine_t *e, aes_stats_t *out)
{
    if (!e || !out)
        return AES_EINVAL;
    e->core.stats(out);
    out->key_hits = e->key_hits.load(std::memory_order_relaxed) - e->key_hits_base;
    out->key_misses = e->key_misses.load(std::memory_order_relaxed) - e->key_misses_base;
    return AES_OK;
}

extern "C" int aes_engine_reset_stats(aes_engine_t *e)
{
    if (!e)
        return AES_EINVAL;
    e->core.reset_stats();
    e->key_hits_base = e->key_hits.load(std::memory_order_relaxed);
    e->key_misses_base = e->key_misses.load(std::memory_order_relaxed);
    return AES_OK;
}

extern "C" uint64_t aes_engine_request_overhead(void)
{
    return sizeof(aesctr::BatchDesc) + sizeof(aesctr::KeyRec);
}

extern "C" int aes_engine_completion_fd(aes_engine_t *e)
{
    if (!e)
        return AES_EINVAL;
    return e->efd >= 0 ? e->efd : AES_EDEVICE;
}
