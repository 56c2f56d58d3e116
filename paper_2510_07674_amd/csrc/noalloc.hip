// Top-M selection without any allocation: spasm_select_topm_static.
//
// The radix-select path of spasm_select_topm_large needs a few tens of KB of device
// scratch (the select state, a 2048-bin histogram, two counts per workgroup range and the
// M selected (key, index) pairs).  Here that scratch is one file-scope device array per
// GPU, sized for the largest supported shape, so the call allocates nothing.
#include <mutex>

#include "spasm_internal.h"

using namespace spasm;

namespace {
// the largest workspace spasm_select_topm_large can ask for: N = 2^20 keys, M = 8192
constexpr size_t TOPM_STATIC_BYTES = 256 + 2048 * sizeof(uint32_t) + 2048 + (size_t)MAX_TOPM_M * 8;

__device__ __align__(256) unsigned char g_topm_scratch[TOPM_STATIC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch[MAX_DEVICES] = {nullptr};

// The device address of this GPU's copy of the scratch array, looked up once per device
// with that device current (in host code the array's name is not a device address).
int scratch_for_current_device(void **out)
{
    int dev = 0;
    SPASM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(SPASM_EUNSUPPORTED, "device %d beyond %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        SPASM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(g_topm_scratch)));
        if (!p) return fail(SPASM_EHIP, "hipGetSymbolAddress returned no address");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return SPASM_OK;
}
}  // namespace

extern "C" size_t spasm_select_topm_static_bytes(void) { return TOPM_STATIC_BYTES; }

extern "C" int spasm_select_topm_static(int32_t N, const float *d_key, int32_t M, int32_t *d_idx, void *stream)
{
    if (N < 1 || N > MAX_TOPM_N) return fail(SPASM_EUNSUPPORTED, "N=%d outside 1..%d", N, MAX_TOPM_N);
    if (M < 1 || M > N) return fail(SPASM_EINVAL, "M=%d outside 1..N", M);
    if (N > MAX_SORT && M > MAX_TOPM_M)
        return fail(SPASM_EUNSUPPORTED, "M=%d above %d for N > %d", M, MAX_TOPM_M, MAX_SORT);
    if (!d_key || !d_idx) return fail(SPASM_EINVAL, "NULL buffer");
    const size_t need = topm_workspace(N, M);
    if (need > TOPM_STATIC_BYTES)
        return fail(SPASM_EUNSUPPORTED, "selection needs %zu bytes of scratch, the static array holds %zu", need,
                    TOPM_STATIC_BYTES);
    int rc = ensure_attrs();
    if (rc) return rc;
    void *scratch = nullptr;
    rc = scratch_for_current_device(&scratch);
    if (rc) return rc;
    // every pass clears or fully writes the scratch it reads (state and histogram are
    // reset by the first kernel, the counts and survivors are written before they are read)
    SPASM_HIP(launch_topm(N, d_key, M, d_idx, scratch, (hipStream_t)stream));
    return SPASM_OK;
}
