// transfer.hip -- data movement around the step: the gather of selected envs
// into a staging block laid out as the public host format (one device-to-host
// copy per field instead of several per env), the library's static staging
// array for callers that cannot allocate, and a plain streaming copy that
// measures the practical HBM ceiling next to the step kernels.
#include <mutex>

#include "device.hpp"
#include "internal.hpp"

namespace gen {

// ---------------------------------------------------------------- env gather
// Workgroup i copies env ids[i] of a batch into row i of each section of the
// staging block (host-format rows of H*W cells, scalars and P general cells
// per env).  All offsets come from GatherArgs, which the host computed with
// gather_layout().
__global__ __launch_bounds__(256) void k_gather_envs(GatherArgs a)
{
    const uint32_t i = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    uint8_t *stg = a.staging;
    const int32_t e = reinterpret_cast<const int32_t *>(stg + a.lay.ids)[i];
    const size_t src0 = (size_t)e * (size_t)a.S, dst0 = (size_t)i * (size_t)a.HW;
    int8_t *owner = reinterpret_cast<int8_t *>(stg + a.lay.owner) + dst0;
    uint8_t *type = stg + a.lay.type + dst0;
    int32_t *army = reinterpret_cast<int32_t *>(stg + a.lay.army) + dst0;
    for (uint32_t c = tid; c < (uint32_t)a.HW; c += blockDim.x) {
        owner[c] = a.owner[src0 + c];
        type[c] = a.type[src0 + c];
        army[c] = a.army[src0 + c];
    }
    if (tid == 0) {
        const EnvScalars s = a.sc[e];
        reinterpret_cast<int32_t *>(stg + a.lay.turn)[i] = s.turn;
        reinterpret_cast<uint32_t *>(stg + a.lay.episode)[i] = s.episode;
        (stg + a.lay.alive)[i] = s.alive;
        (stg + a.lay.finished)[i] = s.finished;
    }
    if (tid < (uint32_t)a.P) reinterpret_cast<int16_t *>(stg + a.lay.gpos)[(size_t)i * a.P + tid] = a.sc[e].gpos[tid];
}

static uint64_t up256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

GatherLayout gather_layout(uint64_t n, uint64_t HW, uint64_t P)
{
    GatherLayout L{};
    uint64_t o = 0;
    L.ids = o;      o += up256(4 * n);
    L.owner = o;    o += up256(n * HW);
    L.type = o;     o += up256(n * HW);
    L.army = o;     o += up256(4 * n * HW);
    L.turn = o;     o += up256(4 * n);
    L.episode = o;  o += up256(4 * n);
    L.alive = o;    o += up256(n);
    L.finished = o; o += up256(n);
    L.gpos = o;     o += up256(2 * n * P);
    L.bytes = o;
    return L;
}

hipError_t launch_gather(const GatherArgs &a, uint32_t n_ids, hipStream_t stream)
{
    hipLaunchKernelGGL(k_gather_envs, dim3(n_ids), dim3(256), 0, stream, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- static staging
// The staging array of gen_get_envs_static: one copy per GPU, alive until
// the process ends.  Host code never uses its name as an address (in host
// code it names a host-side stand-in): the device address comes from
// hipGetSymbolAddress, once per device, with that device current, and only
// that address is passed to kernels and copies.
static __device__ __align__(256) uint8_t scratch[GEN_STATIC_STAGING_BYTES];

namespace {
std::mutex g_sym_mu;
void *g_sym_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_staging(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_sym_mu);
    if (g_sym_ptr[device] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_sym_ptr[device] = p;
    }
    *out = g_sym_ptr[device];
    return hipSuccess;
}

// ---------------------------------------------------------------- streaming copy
// dst[i] = src[i] over 16-byte elements, one element per thread, plain
// loads, nontemporal stores, a grid covering the buffer (no striding loop).  Measured
// against the alternatives (more elements per thread, nontemporal loads,
// a persistent striding grid) it moves the most bytes per second.  A
// measurement of the achievable HBM rate of a read-once / write-once stream.
__global__ __launch_bounds__(256) void k_stream_copy(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src,
                                                      uint64_t n16)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(src[i], dst + i);
}

// dst[i] = src[i / k] (fewer than 2^32 elements): each source element
// written to k consecutive destination elements, in the copy's form; a
// stream that writes k bytes for every byte it reads.  k = 0: zeros, no
// reads (a write-only stream).
__global__ __launch_bounds__(256) void k_stream_spread(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src,
                                                        uint32_t n16, uint32_t k)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(k != 0 ? src[i / k] : u32x4{0u, 0u, 0u, 0u}, dst + i);
}

hipError_t launch_stream_spread(void *dst, const void *src, uint32_t n16, uint32_t k, hipStream_t stream)
{
    const uint32_t grid = (uint32_t)(((uint64_t)n16 + 255) / 256);
    hipLaunchKernelGGL(k_stream_spread, dim3(grid), dim3(256), 0, stream, static_cast<u32x4 *>(dst),
                       static_cast<const u32x4 *>(src), n16, k);
    return hipGetLastError();
}

hipError_t launch_stream_copy(void *dst, const void *src, uint64_t n16, hipStream_t stream)
{
    const uint64_t grid = (n16 + 255) / 256;
    if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3((uint32_t)grid), dim3(256), 0, stream, static_cast<u32x4 *>(dst),
                       static_cast<const u32x4 *>(src), n16);
    return hipGetLastError();
}

}  // namespace gen
