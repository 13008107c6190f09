// api.cpp -- C ABI entry points for single buffers: validation, launch-shape
// resolution and dispatch to the keystream kernels.
#include <mutex>
#include <string.h>

#include "aesctr_internal.h"
#include "tune.h"

namespace aesctr {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_dev_mu;
DeviceInfo g_dev[kMaxDevices];
bool g_dev_ok[kMaxDevices];
thread_local hipError_t t_last_device_error = hipSuccess;

}  // namespace

void note_device_error(hipError_t e)
{
    if (e != hipSuccess)
        t_last_device_error = e;
}

int device_error()
{
    note_device_error(hipGetLastError());
    return AES_EDEVICE;
}

int launch_status()
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        return AES_OK;
    t_last_device_error = e;
    return AES_EDEVICE;
}

int device_info(DeviceInfo *out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        note_device_error(hipGetLastError());
        return AES_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_dev_ok[dev]) {
        DeviceInfo d{};
        d.ordinal = dev;
        if (hipDeviceGetAttribute(&d.num_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipDeviceGetAttribute(&d.max_lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess) {
            note_device_error(hipGetLastError());
            return AES_EDEVICE;
        }
        g_dev[dev] = d;
        g_dev_ok[dev] = true;
    }
    *out = g_dev[dev];
    return AES_OK;
}

int check_sched(const aes_sched_t *s)
{
    if (!s)
        return AES_EINVAL;
    if (!((s->key_bits == 128 && s->nr == 10) || (s->key_bits == 256 && s->nr == 14)))
        return AES_EINVAL;
    return AES_OK;
}

// Argument checks shared by every entry point that takes a buffer pair.
int check_buffers(const void *in, const void *out, uint64_t len)
{
    if (len == 0)
        return AES_OK;
    if (!in || !out)
        return AES_EINVAL;
    if (len > (static_cast<uint64_t>(1) << 36))
        return AES_ERANGE;
    const uintptr_t a = reinterpret_cast<uintptr_t>(in);
    const uintptr_t b = reinterpret_cast<uintptr_t>(out);
    if (a > UINTPTR_MAX - len || b > UINTPTR_MAX - len)
        return AES_EINVAL;
    if (a != b && a < b + len && b < a + len)
        return AES_EOVERLAP;
    return AES_OK;
}

Shape default_shape(int variant, int key_bits, uint64_t len, const DeviceInfo &di)
{
    Shape sh{};
    sh.variant = variant == AES_VARIANT_AUTO ? AES_VARIANT_TTABLE : variant;
    sh.wave_groups = -1;    // first-chunk mode: the rule's (resolve_shape)
    TuneEntry te;
    if (tune_lookup(sh.variant, key_bits, len, &te)) {
        sh.bpl = te.bpl;
        sh.wg = te.wg;
        sh.copies = te.copies;
        sh.tables = te.tables ? te.tables : (te.copies == 64 ? 2 : 4);
        sh.grid = te.grid_per_cu * di.num_cus;
        if (te.first >= kFirstWave0 && te.first <= kFirstFull &&
            first_chunk_mode_ok(te.first, sh.copies, sh.tables, sh.bpl, sh.wg))
            sh.wave_groups = te.first;
    } else if (sh.variant == AES_VARIANT_TTABLE) {
        // The LDS holds only T0 and T2 (32 copies, 64 KiB): half the table
        // fill of four tables, for about 15% more VALU work per block, and
        // room for two workgroups per CU, so one workgroup's fill and
        // barriers overlap the other's keystream.  The chunk a workgroup
        // takes per step (workgroup size x blocks per lane) is the largest
        // that still gives every CU work: a larger chunk leaves CUs idle, a
        // smaller one adds steps.  Measured on MI355X (kernel-only, per
        // launch, against one workgroup per CU with four tables):
        //   AES-128  1 MiB 3.72 us (4.04), 8 MiB 7.84 (8.22), 32 MiB 23.5
        //            (26.6), 256 MiB 172.6 (174.9);
        //   AES-256  1 MiB 4.11 us (4.57, 256 threads), 8 MiB 9.81 (10.19),
        //            32 MiB 30.9 (37.0), 256 MiB 242 (246).
        // Up to 4 MiB one workgroup per CU, each running one chunk, whose
        // rounds 1-2 run in full (first-chunk mode 2: no group constants, no
        // second barrier): 256 threads x 1 block up to 1 MiB, 512 x 1 at
        // 2 MiB, 512 x 2 at 4 MiB.  The autotuner's runs put that 6-10%
        // ahead of 512 threads with wave 0 computing the group constants up
        // to 1 MiB (1 MiB AES-128 3.32 against 3.65 us) and 2-3% at 2-4 MiB.
        // From 8 MiB 512 threads x 2 blocks (x 4 from 16 MiB) with up to
        // four workgroups per CU in the grid, two of them resident at a time.
        sh.grid = di.num_cus;
        sh.copies = 32;
        sh.tables = 2;
        const uint64_t per_cu = (len / 16) / static_cast<uint64_t>(di.num_cus > 0 ? di.num_cus : 1);
        if (per_cu >= 2048) {
            sh.bpl = per_cu >= 4096 ? 4 : 2;
            sh.wg = 512;
            sh.grid = 4 * di.num_cus;
        } else {
            if (per_cu >= 1024) {
                sh.bpl = 2; sh.wg = 512;
            } else if (per_cu >= 512) {
                sh.bpl = 1; sh.wg = 512;
            } else {
                sh.bpl = 1; sh.wg = 256;
            }
            sh.wave_groups = kFirstFull;
        }
    } else if (sh.variant == AES_VARIANT_BITSLICE) {
        sh.bpl = 1;
        sh.wg = 256;
        sh.copies = 0;
        sh.tables = 0;
        sh.grid = 2 * di.num_cus;
    } else {
        // Vector-permute kernel: one block per lane, bound by VALU issue;
        // eight waves per CU keep every SIMD busy.
        sh.bpl = 1;
        sh.wg = 256;
        sh.copies = 0;
        sh.tables = 0;
        sh.grid = 2 * di.num_cus;
    }
    return sh;
}

// Never launch more workgroups than there is work for.
static void clamp_grid(Shape *sh, uint64_t len)
{
    uint64_t blocks = (len + 15) / 16;
    uint64_t per_wg;
    if (sh->variant == AES_VARIANT_BITSLICE)
        per_wg = static_cast<uint64_t>(sh->wg) * 8;    // 512 blocks per wave
    else
        per_wg = static_cast<uint64_t>(sh->wg) * sh->bpl;
    uint64_t need = (blocks + per_wg - 1) / per_wg;
    if (need < 1)
        need = 1;
    if (static_cast<uint64_t>(sh->grid) > need)
        sh->grid = static_cast<int>(need);
}

}  // namespace aesctr

using namespace aesctr;

extern "C" const char *aes_last_device_error(void)
{
    return hipGetErrorName(t_last_device_error);
}

extern "C" const char *aes_strerror(int status)
{
    switch (status) {
    case AES_OK: return "AES_OK: success";
    case AES_EINVAL: return "AES_EINVAL: invalid argument";
    case AES_ENOMEM: return "AES_ENOMEM: out of memory";
    case AES_EAGAIN: return "AES_EAGAIN: over the engine memory budget";
    case AES_ERANGE: return "AES_ERANGE: message longer than 2^32 blocks";
    case AES_EDEVICE: return "AES_EDEVICE: HIP device error or no device";
    case AES_ENOTFOUND: return "AES_ENOTFOUND: unknown ticket";
    case AES_ETIMEDOUT: return "AES_ETIMEDOUT: timed out";
    case AES_EOVERLAP: return "AES_EOVERLAP: input and output partially overlap";
    case AES_ECLOSED: return "AES_ECLOSED: engine is shutting down";
    case AES_ECANCELED: return "AES_ECANCELED: request canceled";
    case AES_ETOOBIG: return "AES_ETOOBIG: more requests than the fixed table holds";
    default: return "unknown aes status";
    }
}

namespace {

int check_cfg(const aes_launch_cfg_t *cfg, int *variant)
{
    *variant = cfg ? cfg->variant : AES_VARIANT_AUTO;
    if (*variant < AES_VARIANT_AUTO || *variant > AES_VARIANT_VPERM)
        return AES_EINVAL;
    if (cfg) {
        if (cfg->blocks_per_lane != 0 && cfg->blocks_per_lane != 1 && cfg->blocks_per_lane != 2 &&
            cfg->blocks_per_lane != 4)
            return AES_EINVAL;
        if (cfg->wg_size != 0 && (cfg->wg_size < 64 || cfg->wg_size > 1024 || cfg->wg_size % 64 != 0))
            return AES_EINVAL;
        if (cfg->grid < 0 || (cfg->lds_copies != 0 && cfg->lds_copies != 32 && cfg->lds_copies != 64))
            return AES_EINVAL;
        if (cfg->lds_tables != 0 && cfg->lds_tables != 2 && cfg->lds_tables != 4)
            return AES_EINVAL;
        if (cfg->lds_copies == 64 && cfg->lds_tables == 4)   // 256 KiB: more than a CU's LDS
            return AES_EINVAL;
        if (cfg->wave_groups < 0 || cfg->wave_groups > 3)
            return AES_EINVAL;
    }
    return AES_OK;
}

// The launch shape for len bytes: the default (or tuned) shape, overridden
// by the non-zero fields of cfg, with the grid clamped to the work.
Shape resolve_shape(int variant, int key_bits, uint64_t len, const aes_launch_cfg_t *cfg, const DeviceInfo &di)
{
    Shape sh = default_shape(variant, key_bits, len, di);
    if (cfg) {
        if (cfg->blocks_per_lane) sh.bpl = cfg->blocks_per_lane;
        if (cfg->wg_size) sh.wg = cfg->wg_size;
        if (cfg->grid) sh.grid = cfg->grid;
        if (cfg->lds_copies) sh.copies = cfg->lds_copies;
        if (cfg->lds_tables) sh.tables = cfg->lds_tables;
    }
    // 64 copies exist only of two tables; a T-table shape always names both.
    if (sh.variant == AES_VARIANT_TTABLE) {
        if (sh.copies == 64)
            sh.tables = 2;
        else if (sh.tables == 0)
            sh.tables = 4;
    }
    if (sh.variant != AES_VARIANT_TTABLE) {
        sh.copies = 0;
        sh.tables = 0;
    }
    if (sh.variant == AES_VARIANT_VPERM)
        sh.bpl = 1;     // one block per lane, whatever cfg asks
    clamp_grid(&sh, len);
    // First-chunk mode of the T-table kernel: cfg's, else the tuned entry's
    // or the rule's (mode 2 up to 4 MiB) where the shape is built for it.
    // Per-wave first-chunk group constants pay off when two workgroups with
    // the 64 KiB image share each CU (8 MiB AES-128: 7.64-7.69 against
    // 7.74-7.78 us); other shapes fall back to wave 0 computing them.
    const int tuned = sh.wave_groups;
    sh.wave_groups = kFirstWave0;
    if (sh.variant == AES_VARIANT_TTABLE) {
        if (cfg && cfg->wave_groups)
            sh.wave_groups = cfg->wave_groups == 3 ? kFirstWave0 : cfg->wave_groups;
        else if (tuned >= 0 && first_chunk_mode_ok(tuned, sh.copies, sh.tables, sh.bpl, sh.wg))
            sh.wave_groups = tuned;
        else if (sh.copies == 32 && sh.tables == 2 && sh.bpl == 2 && sh.wg <= 512 && sh.grid >= 2 * di.num_cus)
            sh.wave_groups = kFirstPerWave;
    }
    return sh;
}

}  // namespace

extern "C" int aes_ctr_launch_shape(int key_bits, size_t len, const aes_launch_cfg_t *cfg, aes_launch_cfg_t *out)
{
    if (!out || (key_bits != 128 && key_bits != 256))
        return AES_EINVAL;
    int variant;
    int rc = check_cfg(cfg, &variant);
    if (rc != AES_OK)
        return rc;
    DeviceInfo di;
    if ((rc = device_info(&di)) != AES_OK)
        return rc;
    const Shape sh = resolve_shape(variant, key_bits, len ? len : 1, cfg, di);
    *out = aes_launch_cfg_t{};
    out->variant = sh.variant;
    out->blocks_per_lane = sh.bpl;
    out->wg_size = sh.wg;
    out->grid = sh.grid;
    out->lds_copies = sh.copies;
    out->lds_tables = sh.tables;
    if (sh.variant == AES_VARIANT_TTABLE &&
        !first_chunk_mode_ok(sh.wave_groups, sh.copies, sh.tables, sh.bpl, sh.wg))
        return AES_EINVAL;
    out->wave_groups = sh.wave_groups;
    return AES_OK;
}

extern "C" int aes_ctr_crypt_cfg(const aes_sched_t *sched, const uint8_t nonce[12], uint32_t ctr0,
                                 const void *in, void *out, size_t len, const aes_launch_cfg_t *cfg,
                                 void *stream)
{
    int rc = check_sched(sched);
    if (rc != AES_OK)
        return rc;
    if (!nonce)
        return AES_EINVAL;
    if ((rc = check_buffers(in, out, len)) != AES_OK)
        return rc;
    int variant;
    if ((rc = check_cfg(cfg, &variant)) != AES_OK)
        return rc;
    if (len == 0)
        return AES_OK;

    DeviceInfo di;
    if ((rc = device_info(&di)) != AES_OK)
        return rc;
    const Shape sh = resolve_shape(variant, sched->key_bits, len, cfg, di);

    hipStream_t st = static_cast<hipStream_t>(stream);
    if (sh.variant == AES_VARIANT_VPERM) {
        VpArgs va;
        make_vperm_args(*sched, nonce, ctr0, in, out, len, &va);
        return launch_ctr_vperm(va, sched->nr, sh, st);
    }
    KeyMaterial km;
    make_key_material(*sched, nonce, &km);
    CtrArgs a{};
    a.in = static_cast<const uint8_t *>(in);
    a.out = static_cast<uint8_t *>(out);
    a.len = len;
    a.ctr0 = ctr0;
    a.x0 = km.x0;
    memcpy(a.k1, km.k1, sizeof(a.k1));
    memcpy(a.rk, km.rk, sizeof(a.rk));
    if (sh.variant == AES_VARIANT_BITSLICE)
        return launch_ctr_bitslice(a, km.nr, sh, st);
    return launch_ctr_ttable(a, km.nr, sh, st);
}

extern "C" int aes_ctr_crypt(const aes_sched_t *sched, const uint8_t nonce[12], uint32_t ctr0,
                             const void *in, void *out, size_t len, void *stream)
{
    return aes_ctr_crypt_cfg(sched, nonce, ctr0, in, out, len, nullptr, stream);
}
