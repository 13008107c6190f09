// roofline_probe.hip -- measures the MI355X ceilings the AES kernels are
// held against: random 4-byte LDS reads per clock and CU (the T-table
// kernels' bound) for several bank-replication layouts, 32-bit VALU issue
// rate, HBM copy bandwidth, the per-launch floor of back-to-back kernels
// (graph-replayed and eager), and pinned PCIe copies.  Prints one JSON object
// per measurement.
//
// Usage: roofline_probe
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <vector>

#define CK(x)                                                                                  \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) {                                                                \
            fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);     \
            exit(1);                                                                           \
        }                                                                                      \
    } while (0)

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// Pointer chase through 128 KiB of LDS: each loaded word is the next byte
// address (row x at 256*x, the lane's slot at +4*slot), 8 independent chains
// per lane, so no VALU work sits between lookups.  SLOTS = number of distinct
// bank slots lanes spread over (64, 32, 16 or 1).
template <int SLOTS, bool PERM>
__global__ __launch_bounds__(1024) void lds_chase(uint32_t *out, int iters)
{
    __shared__ uint32_t lds[32768];
    for (int w = threadIdx.x; w < 32768; w += blockDim.x) {
        const uint32_t row = (w >> 6) & 255, k = w & 63;
        lds[w] = ((mix32(row * 7919u + (w >> 14)) & 0xffu) << 8) | (k * 4);
    }
    __syncthreads();
    const uint32_t slot = (threadIdx.x & 63) % SLOTS;
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        v[j] = ((mix32(threadIdx.x * 131 + j) & 0xff) << 8) | (slot * 4);
    const char *base = reinterpret_cast<const char *>(lds);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            uint32_t a = v[j];
            if (PERM)
                a = __builtin_amdgcn_perm(a, slot * 4, 0x0c020500u);   // as the cipher builds addresses
            v[j] = *reinterpret_cast<const uint32_t *>(base + a);
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) r += v[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// 8 independent chains of 3-input boolean ops (v_bitop3_b32).
__global__ __launch_bounds__(1024) void valu_chain(uint32_t *out, int iters)
{
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = mix32(threadIdx.x * 8 + j);
    const uint32_t k = mix32(blockIdx.x);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = __builtin_amdgcn_bitop3_b32(v[j], v[(j + 1) & 7], k, 0x96);
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) r ^= v[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

__global__ void copy_kernel(const u32x4 *__restrict__ in, u32x4 *__restrict__ out, size_t n)
{
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(in + i), out + i);
}

__global__ void empty_kernel(int *p)
{
    if (p && threadIdx.x == 1u << 20)
        p[0] = 1;
}

struct Timer {
    hipEvent_t a, b;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st)
    {
        CK(hipEventCreate(&a));
        CK(hipEventCreate(&b));
    }
    void start() { CK(hipEventRecord(a, s)); }
    float stop_ms()
    {
        CK(hipEventRecord(b, s));
        CK(hipEventSynchronize(b));
        float ms;
        CK(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
};

}  // namespace

int main()
{
    CK(hipSetDevice(0));
    hipDeviceProp_t p;
    CK(hipGetDeviceProperties(&p, 0));
    const int cus = p.multiProcessorCount;
    const double clk = p.clockRate * 1e3;   // Hz (peak engine clock)
    printf("{\"probe\": \"device\", \"name\": \"%s\", \"arch\": \"%s\", \"cus\": %d, \"clock_hz\": %.0f, "
           "\"lds_per_block\": %zu, \"l2_bytes\": %d}\n",
           p.name, p.gcnArchName, cus, clk, p.sharedMemPerBlock, p.l2CacheSize);
    hipStream_t s;
    CK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    Timer t(s);
    uint32_t *out;
    CK(hipMalloc(&out, static_cast<size_t>(cus) * 4 * 1024 * sizeof(uint32_t)));   // largest grid: 4 * cus x 1024

    struct L {
        const char *name;
        void (*k)(uint32_t *, int);
    } lds_cases[] = {
        {"64 slots (lane)", lds_chase<64, false>},
        {"32 slots (lane mod 32)", lds_chase<32, false>},
        {"16 slots (lane mod 16)", lds_chase<16, false>},
        {"1 slot (all lanes one bank)", lds_chase<1, false>},
        {"64 slots + one v_perm_b32 per lookup", lds_chase<64, true>},
    };
    for (auto &c : lds_cases) {
        const int iters = 4096;
        hipLaunchKernelGGL(c.k, dim3(cus), dim3(1024), 0, s, out, 16);
        t.start();
        hipLaunchKernelGGL(c.k, dim3(cus), dim3(1024), 0, s, out, iters);
        const float ms = t.stop_ms();
        const double n = static_cast<double>(cus) * 1024 * iters * 8;
        printf("{\"probe\": \"lds_random_read_b32\", \"layout\": \"%s\", \"lookups_per_clk_per_cu\": %.2f, "
               "\"bytes_per_clk_per_cu\": %.1f, \"ms\": %.3f}\n",
               c.name, n / (ms * 1e-3) / cus / clk, 4 * n / (ms * 1e-3) / cus / clk, ms);
    }
    {
        const int iters = 8192;
        hipLaunchKernelGGL(valu_chain, dim3(cus * 4), dim3(1024), 0, s, out, 16);
        t.start();
        hipLaunchKernelGGL(valu_chain, dim3(cus * 4), dim3(1024), 0, s, out, iters);
        const float ms = t.stop_ms();
        const double n = static_cast<double>(cus) * 4 * 1024 * iters * 8;
        printf("{\"probe\": \"valu_bitop3\", \"lane_ops_per_clk_per_cu\": %.2f, \"ms\": %.3f}\n",
               n / (ms * 1e-3) / cus / clk, ms);
    }
    // HBM: 1 GiB copy, and 8 MiB copies rotating over 768 MiB.
    const size_t big = static_cast<size_t>(1) << 30;
    u32x4 *a, *b;
    CK(hipMalloc(&a, big));
    CK(hipMalloc(&b, big));
    CK(hipMemset(a, 1, big));
    CK(hipMemset(b, 0, big));
    for (int grid : {cus * 4, cus * 8}) {
        hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, s, a, b, big / 16);
        t.start();
        hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, s, a, b, big / 16);
        const float ms = t.stop_ms();
        printf("{\"probe\": \"hbm_copy\", \"bytes\": %zu, \"grid\": %d, \"read_plus_write_gbs\": %.1f}\n", big,
               grid, 2.0 * big / ms / 1e6);
    }
    auto graph_floor = [&](const char *name, auto launch) {
        const int n = 1000;
        hipGraph_t g;
        hipGraphExec_t ge;
        CK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < n; ++i) launch(i);
        CK(hipStreamEndCapture(s, &g));
        CK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        CK(hipGraphLaunch(ge, s));
        CK(hipStreamSynchronize(s));
        t.start();
        CK(hipGraphLaunch(ge, s));
        const float gms = t.stop_ms();
        t.start();
        for (int i = 0; i < n; ++i) launch(i);
        const float ems = t.stop_ms();
        printf("{\"probe\": \"back_to_back_launch\", \"kernel\": \"%s\", \"graph_us_per_launch\": %.3f, "
               "\"eager_us_per_launch\": %.3f}\n",
               name, gms * 1e3 / n, ems * 1e3 / n);
        CK(hipGraphExecDestroy(ge));
        CK(hipGraphDestroy(g));
    };
    graph_floor("empty 256x1024", [&](int) { hipLaunchKernelGGL(empty_kernel, dim3(256), dim3(1024), 0, s, nullptr); });
    const size_t m8 = 8 << 20;
    graph_floor("copy 8 MiB (rotating over 768 MiB)", [&](int i) {
        const size_t off = (static_cast<size_t>(i) % 48) * m8 / 16;
        hipLaunchKernelGGL(copy_kernel, dim3(cus * 4), dim3(256), 0, s, a + off, b + off, m8 / 16);
    });
    // PCIe, pinned host memory.
    void *h;
    const size_t hb = 256 << 20;
    CK(hipHostMalloc(&h, hb, hipHostMallocDefault));
    for (int dir = 0; dir < 2; ++dir) {
        for (int rep = 0; rep < 2; ++rep) {
            t.start();
            if (dir == 0)
                CK(hipMemcpyAsync(a, h, hb, hipMemcpyHostToDevice, s));
            else
                CK(hipMemcpyAsync(h, a, hb, hipMemcpyDeviceToHost, s));
            const float ms = t.stop_ms();
            if (rep)
                printf("{\"probe\": \"pcie_pinned\", \"direction\": \"%s\", \"gbs\": %.1f}\n", dir ? "D2H" : "H2D",
                       hb / ms / 1e6);
        }
    }
    CK(hipHostFree(h));
    CK(hipFree(a));
    CK(hipFree(b));
    CK(hipFree(out));
    return 0;
}
