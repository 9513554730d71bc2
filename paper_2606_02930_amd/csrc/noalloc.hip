// Fixed per-device working memory for the entry point that allocates nothing
// (ite_mps_sample_noalloc).  The array below is reserved on every GPU the
// library runs on, for the life of the process.  Host code never uses its
// name as an address: its device address is looked up once per device, with
// that device current, when the first context on it is created, and that
// address is what the kernels receive.
#include "engine.h"

#include <mutex>

namespace {

constexpr size_t SCRATCH_BYTES = 64ull << 20;   // 64 MiB per GPU
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) double scratch[SCRATCH_BYTES / sizeof(double)];

std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

}  // namespace

namespace ite {

size_t noalloc_scratch_doubles() { return SCRATCH_BYTES / sizeof(double); }

// Looks up this device's copy of the scratch array (the device must be
// current).  Idempotent; thread-safe.
void noalloc_init(int device) {
    ITE_REQUIRE(device >= 0 && device < MAX_DEVICES, "noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return;
    void* p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) ITE_FAIL(ITE_EDEVICE, "noalloc: no device address for the scratch array");
    g_ptr[device] = static_cast<double*>(p);
}

// Device address of `device`'s scratch array (looked up on first use when no
// context was created on that device yet; the device must be current).
double* noalloc_scratch(int device) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (device >= 0 && device < MAX_DEVICES && g_ptr[device]) return g_ptr[device];
    }
    noalloc_init(device);
    return g_ptr[device];
}

}  // namespace ite
