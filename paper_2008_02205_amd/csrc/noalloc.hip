// Overlap lists without any allocation: the cell-list search of
// mlpg_neighbors_count / mlpg_neighbors_fill with its scratch (bounding box,
// each point's cell, cell counts and starts, points in cell order) in a
// file-scope device array instead of memory the library allocates.  For
// callers that cannot allocate device memory while they run.
#include <mutex>

#include "internal.hpp"

namespace mlpg {

namespace {

constexpr int64_t kStaticPoints = (int64_t)1 << 20;   // most points per call
constexpr int64_t kStaticCells = (int64_t)1 << 20;    // grid cells of the search

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// the layout of nb_scratch_at(ptr, kStaticPoints, kStaticCells)
constexpr size_t kStaticBytes = align256(8 * 8) + align256(4 * (size_t)kStaticPoints) +
                                align256(4 * (size_t)kStaticCells) + align256(8 * (size_t)(kStaticCells + 1)) +
                                align256(4 * (size_t)kStaticPoints);

// One copy per GPU, held until the process ends.  In host code the name is
// only a stand-in: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

// The current device's copy of the array (looked up once per device).
int scratch_ptr(void **out)
{
    int dev = -1;
    MLPG_HIP(hipGetDevice(&dev));
    MLPG_CHECK(dev >= 0 && dev < kMaxDevices, MLPG_ERR_ARG, "mlpg_neighbors_static: device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        MLPG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        MLPG_CHECK(p != nullptr, MLPG_ERR_HIP, "mlpg_neighbors_static: no device address for the scratch array");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return MLPG_OK;
}

}  // namespace

}  // namespace mlpg

using namespace mlpg;

extern "C" int mlpg_neighbors_static(int dim, int64_t n, const double *x, const double *R, int64_t *nbr_off,
                                     int32_t *nbr_idx, int64_t cap, int64_t *total, void *stream)
{
    MLPG_CHECK(dim == 2 || dim == 3, MLPG_ERR_ARG, "mlpg_neighbors_static: dim must be 2 or 3");
    MLPG_CHECK(n > 0 && n <= kStaticPoints, MLPG_ERR_ARG,
               "mlpg_neighbors_static: n must be in [1, " + std::to_string(kStaticPoints) +
                   "] (the size of the static scratch)");
    MLPG_CHECK(x && R && nbr_off && total && cap >= 0 && (cap == 0 || nbr_idx), MLPG_ERR_ARG,
               "mlpg_neighbors_static: null pointer or negative capacity");
    void *base = nullptr;
    int rc = scratch_ptr(&base);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const NbScratch sc = nb_scratch_at(base, kStaticPoints, kStaticCells);
    // counts into nbr_off, scanned in place (every scratch entry the search
    // reads is written by it first; the cell counts are cleared by a kernel)
    MLPG_HIP(launch_neighbors_count(dim, n, x, R, nbr_off, sc, s));
    MLPG_HIP(launch_exclusive_scan(nbr_off, nbr_off, n, s));
    int64_t tot = 0;
    MLPG_HIP(hipMemcpyAsync(&tot, nbr_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MLPG_HIP(hipStreamSynchronize(s));
    *total = tot;
    if (tot > cap) {
        set_error("mlpg_neighbors_static: " + std::to_string(tot) + " list entries, capacity " + std::to_string(cap));
        return MLPG_ERR_CAPACITY;
    }
    if (tot > 0) {
        MLPG_HIP(launch_neighbors_fill(dim, n, x, R, nbr_off, nbr_idx, sc, s));
        MLPG_HIP(hipStreamSynchronize(s));
    }
    return MLPG_OK;
}
