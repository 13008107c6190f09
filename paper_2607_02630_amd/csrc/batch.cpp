// batch.cpp -- aes_ctr_crypt_batch: descriptor table staging and the
// captured-graph launch.
//
// Per (device, stream) the library keeps a context: a device table (header +
// up to kMaxBatch descriptors, their inline keys and key installs) and a ring
// of pinned host staging slots, each with an executable HIP graph of two
// nodes -- the host-to-device copy of that slot into the table, then the
// persistent batch kernel.  A call fills a free slot, sets its graph's copy
// size, and launches the graph on the caller's stream; nothing is
// re-captured between calls.  A slot (and its graph) is reused only after the
// event recorded behind its last launch completes, so no update touches a
// graph still in flight.  The tile counter the kernel claims work from is
// part of every upload (0), so no memset node is needed.  The call cannot
// itself be captured into a caller's graph (its staging would be rewritten
// by later calls): on a capturing stream it returns AES_EINVAL.
#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string.h>
#include <vector>

#include "aesctr_internal.h"
#include "host_pool.h"
#include "tune.h"

namespace aesctr {

namespace {

constexpr int kSlots = 4;
constexpr size_t kTableBytes = kMaxTableBytes;

// Descriptors per part of the host's parallel validation.
constexpr size_t kCheckGrain = 4096;

struct BatchShape {
    int tile_bytes, wg, grid, bpl, use_graph;
};

struct SlotGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy_node = nullptr;
    int grid = 0, bpl = 0;
};

struct BatchCtx {
    std::mutex mu;
    int device = -1;
    void *dev_table = nullptr;
    uint8_t *staging[kSlots] = {};
    hipEvent_t done[kSlots] = {};
    bool used[kSlots] = {};
    SlotGraph g[kSlots];
    int next_slot = 0;
};

std::mutex g_ctx_mu;
// Contexts live until process exit (freeing them from a static destructor
// could run after the HIP runtime has shut down).  A stream's context goes
// back to its device's free list when the stream is retired
// (release_batch_stream, called by aes_engine_destroy before it destroys its
// streams), and the next new stream on that device takes it over, so
// creating and destroying engines does not grow memory.
std::map<std::pair<int, void *>, BatchCtx *> g_ctx;
std::map<int, std::vector<BatchCtx *>> g_free;

int init_ctx(BatchCtx *c, int device)
{
    c->device = device;
    if (hipMalloc(&c->dev_table, kTableBytes) != hipSuccess)
        return AES_ENOMEM;
    for (int i = 0; i < kSlots; ++i) {
        if (hipHostMalloc(reinterpret_cast<void **>(&c->staging[i]), kTableBytes, hipHostMallocDefault) !=
            hipSuccess)
            return AES_ENOMEM;
        if (hipEventCreateWithFlags(&c->done[i], hipEventDisableTiming) != hipSuccess)
            return AES_EDEVICE;
    }
    return AES_OK;
}

BatchCtx *get_ctx(int device, void *stream, int *rc)
{
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    auto key = std::make_pair(device, stream);
    auto it = g_ctx.find(key);
    if (it != g_ctx.end()) {
        *rc = AES_OK;
        return it->second;
    }
    std::vector<BatchCtx *> &fl = g_free[device];
    if (!fl.empty()) {
        BatchCtx *c = fl.back();
        fl.pop_back();
        g_ctx[key] = c;
        *rc = AES_OK;
        return c;
    }
    BatchCtx *c = new BatchCtx();
    *rc = init_ctx(c, device);
    if (*rc != AES_OK) {
        note_device_error(hipGetLastError());
        return nullptr;   // partially initialised context is leaked deliberately
    }
    g_ctx[key] = c;
    return c;
}

// Capture (copy of slot s into the table) + kernel on a private stream.
int build_graph(BatchCtx *c, int s, int grid, int bpl)
{
    SlotGraph &sg = c->g[s];
    if (sg.exec) {
        (void)hipGraphExecDestroy(sg.exec);
        (void)hipGraphDestroy(sg.graph);
        sg = SlotGraph{};
    }
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
        return AES_EDEVICE;
    int rc = AES_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = AES_EDEVICE;
    } else {
        (void)hipMemcpyAsync(c->dev_table, c->staging[s], kTableBytes, hipMemcpyHostToDevice, cap);
        int lrc = launch_ctr_batch(c->dev_table, grid, 1024, bpl, cap);
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(cap, &g) != hipSuccess || lrc != AES_OK || !g) {
            rc = lrc != AES_OK ? lrc : AES_EDEVICE;
        } else {
            sg.graph = g;
            size_t nn = 0;
            (void)hipGraphGetNodes(g, nullptr, &nn);
            std::vector<hipGraphNode_t> nodes(nn);
            (void)hipGraphGetNodes(g, nodes.data(), &nn);
            for (hipGraphNode_t nd : nodes) {
                hipGraphNodeType ty;
                if (hipGraphNodeGetType(nd, &ty) == hipSuccess && ty == hipGraphNodeTypeMemcpy)
                    sg.copy_node = nd;
            }
            if (!sg.copy_node || hipGraphInstantiate(&sg.exec, g, nullptr, nullptr, 0) != hipSuccess)
                rc = AES_EDEVICE;
        }
    }
    (void)hipStreamDestroy(cap);
    if (rc != AES_OK) {
        note_device_error(hipGetLastError());
        sg.exec = nullptr;
        return rc;
    }
    sg.grid = grid;
    sg.bpl = bpl;
    return AES_OK;
}

}  // namespace

// Completes a staged table at buf: n descriptors, header.n_keys inline keys
// and header.n_install installs written.  Assigns first tiles and fills the
// rest of the header.  Returns the bytes to upload, or 0 if the tile count
// would overflow.
size_t finish_stage(uint8_t *buf, size_t n, uint32_t tile_blocks)
{
    BatchHeader *h = reinterpret_cast<BatchHeader *>(buf);
    BatchDesc *out = reinterpret_cast<BatchDesc *>(buf + sizeof(BatchHeader));
    uint64_t tiles = 0;
    for (size_t i = 0; i < n; ++i) {
        out[i].tile0 = static_cast<uint32_t>(tiles);
        const uint64_t blocks = (out[i].len + 15) / 16;
        tiles += (blocks + tile_blocks - 1) / tile_blocks;
        if (tiles > 0x7fffffffu)
            return 0;
    }
    h->n = static_cast<uint32_t>(n);
    h->total_tiles = static_cast<uint32_t>(tiles);
    h->tile_blocks = tile_blocks;
    h->next = 0;
    h->keys_off = static_cast<uint32_t>(batch_keys_off(n));
    h->install_off = static_cast<uint32_t>(batch_install_off(n, h->n_keys));
    memset(h->pad, 0, sizeof(h->pad));
    return batch_table_bytes(n, h->n_keys, h->n_install);
}

namespace {

// Records per part of the host's parallel record building.
constexpr size_t kRecordGrain = 256;

// A batch of at most kSmallBatch requests goes in the kernel's argument block
// (no staging slot, no upload).  Its kernel has four waves per workgroup and
// sizes its own grid: a wave per tile, at most two workgroups per CU of the
// table kernel's grid (which is at most one per CU), the waves looping over
// further tiles.  Returns AES_OK, AES_ERANGE or AES_EDEVICE.
int launch_small(hipStream_t st, const LaunchSpec &spec, uint32_t tile_blocks, int grid, int bpl)
{
    SmallBatchArgs args{};
    uint64_t tiles = 0;
    for (size_t i = 0; i < spec.n; ++i) {
        const BatchDesc &d = spec.descs[i];
        SmallRec &r = args.r[i];
        r.in = d.in;
        r.out = d.out;
        r.len = d.len;
        r.ctr0 = d.ctr0;
        r.x0 = d.x0;
        r.nr = d.nr;
        r.aligned = d.aligned;
        memcpy(r.k1, d.k1, sizeof(r.k1));
        r.key = d.key;
        r.install = kNoInstall;
        if (!(d.key & kKeyResident)) {
            memcpy(r.rk, spec.keys[d.key].rk, sizeof(r.rk));
            for (size_t j = 0; j < spec.n_install; ++j)
                if (spec.installs[j].key == d.key)
                    r.install = spec.installs[j].slot;
        }
        r.tile0 = static_cast<uint32_t>(tiles);
        tiles += ((d.len + 15) / 16 + tile_blocks - 1) / tile_blocks;
        if (tiles > 0x7fffffffu)
            return AES_ERANGE;
    }
    // An install names one inline key; two records sharing that key must not
    // both write the slot: keep the first.
    for (size_t i = 0; i < spec.n; ++i)
        for (size_t j = 0; j < i; ++j)
            if (args.r[i].install != kNoInstall && args.r[i].install == args.r[j].install)
                args.r[i].install = kNoInstall;
    args.n = static_cast<uint32_t>(spec.n);
    args.total_tiles = static_cast<uint32_t>(tiles);
    args.tile_blocks = tile_blocks;
    args.resident = spec.resident;
    const uint64_t want = (tiles + 3) / 4;
    const uint64_t cap = 2 * static_cast<uint64_t>(grid);
    const int small_grid = static_cast<int>(std::max<uint64_t>(1, std::min(want, cap)));
    return launch_ctr_batch_small(args, small_grid, bpl, st);
}

// Takes the context's next staging slot once its last launch has finished.
int take_slot(BatchCtx *c, int *slot)
{
    *slot = c->next_slot;
    c->next_slot = (c->next_slot + 1) % kSlots;
    if (c->used[*slot] && hipEventSynchronize(c->done[*slot]) != hipSuccess) {
        note_device_error(hipGetLastError());
        return AES_EDEVICE;
    }
    return AES_OK;
}

// Uploads the first `bytes` of staging slot `slot` into the device table and
// launches the batch kernel on st, through the slot's captured graph or a
// plain copy + launch, then marks the slot busy until that work finishes.
int submit_slot(BatchCtx *c, int slot, size_t bytes, hipStream_t st, int grid, int bpl, bool use_graph)
{
    int rc;
    if (use_graph) {
        SlotGraph &sg = c->g[slot];
        if (!sg.exec || sg.grid != grid || sg.bpl != bpl) {
            if ((rc = build_graph(c, slot, grid, bpl)) != AES_OK)
                return rc;
        }
        if (hipGraphExecMemcpyNodeSetParams1D(sg.exec, sg.copy_node, c->dev_table, c->staging[slot], bytes,
                                              hipMemcpyHostToDevice) != hipSuccess ||
            hipGraphLaunch(sg.exec, st) != hipSuccess) {
            note_device_error(hipGetLastError());
            return AES_EDEVICE;
        }
    } else {
        if (hipMemcpyAsync(c->dev_table, c->staging[slot], bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
            note_device_error(hipGetLastError());
            return AES_EDEVICE;
        }
        if ((rc = launch_ctr_batch(c->dev_table, grid, 1024, bpl, st)) != AES_OK)
            return rc;
    }
    if (hipEventRecord(c->done[slot], st) != hipSuccess) {
        note_device_error(hipGetLastError());
        return AES_EDEVICE;
    }
    c->used[slot] = true;
    return AES_OK;
}

}  // namespace

int launch_spec(int device, hipStream_t st, const LaunchSpec &spec, int tile_bytes, int grid, int bpl,
                bool use_graph, bool allow_small)
{
    const uint32_t tile_blocks = static_cast<uint32_t>(tile_bytes / 16);
    if (spec.n == 0)
        return AES_OK;
    if (spec.n > static_cast<size_t>(kMaxBatch) || spec.n_keys > static_cast<size_t>(kMaxBatch) ||
        spec.n_install > static_cast<size_t>(kMaxBatch))
        return AES_EINVAL;
    if (allow_small && spec.n <= kSmallBatch)
        return launch_small(st, spec, tile_blocks, grid, bpl);
    int rc;
    BatchCtx *c = get_ctx(device, st, &rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    int slot;
    if ((rc = take_slot(c, &slot)) != AES_OK)
        return rc;
    uint8_t *buf = c->staging[slot];
    BatchHeader *h = reinterpret_cast<BatchHeader *>(buf);
    memset(h, 0, sizeof(*h));
    h->n_keys = static_cast<uint32_t>(spec.n_keys);
    h->n_install = static_cast<uint32_t>(spec.n_install);
    h->resident = spec.resident;
    memcpy(buf + sizeof(BatchHeader), spec.descs, spec.n * sizeof(BatchDesc));
    memcpy(buf + batch_keys_off(spec.n), spec.keys, spec.n_keys * sizeof(KeyRec));
    memcpy(buf + batch_install_off(spec.n, spec.n_keys), spec.installs, spec.n_install * sizeof(InstallRec));
    const size_t bytes = finish_stage(buf, spec.n, tile_blocks);
    if (bytes == 0)
        return AES_ERANGE;
    return submit_slot(c, slot, bytes, st, grid, bpl, use_graph);
}

void release_batch_stream(int device, hipStream_t st)
{
    BatchCtx *c = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        auto it = g_ctx.find(std::make_pair(device, static_cast<void *>(st)));
        if (it == g_ctx.end())
            return;
        c = it->second;
        g_ctx.erase(it);
    }
    {
        // The stream's last launches read the staging slots: wait for them
        // before another stream may refill a slot.
        std::lock_guard<std::mutex> lk(c->mu);
        for (int i = 0; i < kSlots; ++i) {
            if (c->used[i] && hipEventSynchronize(c->done[i]) != hipSuccess)
                note_device_error(hipGetLastError());
            c->used[i] = false;
        }
    }
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    g_free[device].push_back(c);
}

uint64_t batch_tile_bytes(uint64_t batch_bytes, int num_cus)
{
    // About kTilesPerCu tiles per CU (one per wave of a workgroup), between
    // 2 KiB (one wave step: 64 lanes x 2 blocks) and kMaxTile, multiples of
    // 2 KiB; the tune cache's batch entry may set both constants.  Measured on
    // MI355X: on the 4096-request workload 64 KiB tiles (3.59 ms) beat 16 KiB
    // (3.67) and 4 KiB (12.8, when every tile was claimed with an atomic);
    // small batches need small tiles to reach many CUs.
    constexpr uint64_t kTilesPerCu = 16, kMaxTile = 65536;
    uint64_t tpc = kTilesPerCu, max_tile = kMaxTile;
    TuneEntry te;
    if (tune_lookup_batch(&te)) {
        if (te.tiles_per_cu >= 1 && te.tiles_per_cu <= 1024)
            tpc = static_cast<uint64_t>(te.tiles_per_cu);
        if (te.max_tile_bytes >= 2048 && te.max_tile_bytes <= (1 << 24) && te.max_tile_bytes % 2048 == 0)
            max_tile = static_cast<uint64_t>(te.max_tile_bytes);
    }
    const uint64_t cus = static_cast<uint64_t>(num_cus > 0 ? num_cus : 1);
    uint64_t tile = (batch_bytes / (tpc * cus) + 2047) & ~uint64_t(2047);
    return tile < 2048 ? 2048 : tile > max_tile ? max_tile : tile;
}

int batch_blocks_per_lane()
{
    TuneEntry te;
    return tune_lookup_batch(&te) && (te.bpl == 1 || te.bpl == 2) ? te.bpl : 2;
}

// Descriptor (key field left 0) and round keys of one validated request.
void make_batch_desc(const aes_ctr_desc_t &d, BatchDesc *o, KeyRec *k)
{
    KeyMaterial km;
    make_key_material(*d.sched, d.nonce, &km);
    memset(o, 0, sizeof(*o));
    o->in = reinterpret_cast<uint64_t>(d.in);
    o->out = reinterpret_cast<uint64_t>(d.out);
    o->len = d.len;
    o->ctr0 = d.ctr0;
    o->x0 = km.x0;
    o->nr = static_cast<uint16_t>(km.nr);
    o->aligned = ((o->in | o->out) & 15) == 0;
    memcpy(o->k1, km.k1, sizeof(o->k1));
    memset(k, 0, sizeof(*k));
    memcpy(k->rk, km.rk, sizeof(km.rk));
}

void make_batch_record(const aes_ctr_desc_t &d, RequestRec *o)
{
    make_batch_desc(d, &o->d, &o->key);
}

int check_desc(const aes_ctr_desc_t &d)
{
    int rc = check_sched(d.sched);
    if (rc != AES_OK)
        return rc;
    if (d.flags != 0)
        return AES_EINVAL;
    return check_buffers(d.in, d.out, d.len);
}

}  // namespace aesctr

using namespace aesctr;

extern "C" int aes_ctr_crypt_batch_cfg(const aes_ctr_desc_t *desc, size_t n, const aes_batch_cfg_t *cfg,
                                       void *stream)
{
    if (n == 0)
        return AES_OK;
    if (!desc)
        return AES_EINVAL;
    // Validation and the payload total, over parts in parallel; the status of
    // the first failing descriptor wins, as in a serial scan.
    struct Scan {
        int rc;
        uint64_t bytes;
    };
    const size_t parts = HostPool::parts(n, kCheckGrain);
    Scan scan[HostPool::kMaxParts];
    HostPool::get().parallel_for(n, kCheckGrain, [&](size_t p, size_t b, size_t e) {
        Scan r{AES_OK, 0};
        for (size_t i = b; i < e && r.rc == AES_OK; ++i) {
            r.rc = check_desc(desc[i]);
            r.bytes += desc[i].len;
        }
        scan[p] = r;
    });
    uint64_t total_bytes = 0;
    for (size_t p = 0; p < parts; ++p) {
        if (scan[p].rc != AES_OK)
            return scan[p].rc;
        total_bytes += scan[p].bytes;
    }
    // Tile size 0 = sized to the batch (batch_tile_bytes); two blocks per
    // lane unless the tune cache says otherwise.
    BatchShape sh{0, 1024, 0, batch_blocks_per_lane(), 1};
    if (cfg) {
        if (cfg->tile_bytes < 0 || (cfg->tile_bytes && (cfg->tile_bytes % 1024 != 0 || cfg->tile_bytes > (1 << 26))))
            return AES_EINVAL;
        if (cfg->wg_size != 0 && cfg->wg_size != 1024)
            return AES_EINVAL;
        if (cfg->grid < 0 || cfg->grid > kMaxBatchGrid ||
            (cfg->blocks_per_lane != 0 && cfg->blocks_per_lane != 1 && cfg->blocks_per_lane != 2))
            return AES_EINVAL;
        if (cfg->tile_bytes) sh.tile_bytes = cfg->tile_bytes;
        if (cfg->grid) sh.grid = cfg->grid;
        if (cfg->blocks_per_lane) sh.bpl = cfg->blocks_per_lane;
        sh.use_graph = cfg->use_graph;
    }
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != AES_OK)
        return rc;
    if (sh.grid == 0)
        sh.grid = di.num_cus;

    hipStream_t st = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        note_device_error(hipGetLastError());
        return AES_EDEVICE;
    }
    if (cs != hipStreamCaptureStatusNone)
        return AES_EINVAL;

    if (sh.tile_bytes == 0)
        sh.tile_bytes = static_cast<int>(batch_tile_bytes(total_bytes, di.num_cus));
    const uint32_t tile_blocks = static_cast<uint32_t>(sh.tile_bytes / 16);

    // At most kSmallBatch requests: records in the kernel arguments.
    if (n <= kSmallBatch) {
        BatchDesc descs[kSmallBatch];
        KeyRec keys[kSmallBatch];
        for (size_t i = 0; i < n; ++i) {
            make_batch_desc(desc[i], &descs[i], &keys[i]);
            descs[i].key = static_cast<uint32_t>(i);
        }
        LaunchSpec spec;
        spec.descs = descs;
        spec.n = n;
        spec.keys = keys;
        spec.n_keys = n;
        return launch_small(st, spec, tile_blocks, sh.grid, sh.bpl);
    }

    // Otherwise launches of up to kMaxBatch requests, each request's key
    // inline.  Records are built straight into the pinned staging slot.
    BatchCtx *c = get_ctx(di.ordinal, st, &rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    for (size_t first = 0; first < n; first += kMaxBatch) {
        const size_t m = n - first < static_cast<size_t>(kMaxBatch) ? n - first : kMaxBatch;
        int slot;
        if ((rc = take_slot(c, &slot)) != AES_OK)
            return rc;
        uint8_t *buf = c->staging[slot];
        BatchHeader *h = reinterpret_cast<BatchHeader *>(buf);
        memset(h, 0, sizeof(*h));
        h->n_keys = static_cast<uint32_t>(m);
        BatchDesc *out = reinterpret_cast<BatchDesc *>(buf + sizeof(BatchHeader));
        KeyRec *keys = reinterpret_cast<KeyRec *>(buf + batch_keys_off(m));
        HostPool::get().parallel_for(m, kRecordGrain, [&](size_t, size_t b, size_t e) {
            for (size_t i = b; i < e; ++i) {
                make_batch_desc(desc[first + i], out + i, keys + i);
                out[i].key = static_cast<uint32_t>(i);
            }
        });
        const size_t bytes = finish_stage(buf, m, tile_blocks);
        if (bytes == 0)
            return AES_ERANGE;
        if ((rc = submit_slot(c, slot, bytes, st, sh.grid, sh.bpl, sh.use_graph != 0)) != AES_OK)
            return rc;
    }
    return AES_OK;
}

extern "C" int aes_ctr_crypt_batch(const aes_ctr_desc_t *desc, size_t n, void *stream)
{
    return aes_ctr_crypt_batch_cfg(desc, n, nullptr, stream);
}
