// Allocation-free point binning: mot_bin_points for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// The two temporaries of the binning -- each point's tile id and the 64-bit sort keys of
// the bitonic stable sort -- live in one file-scope device array instead of per-call
// hipMalloc buffers; the cells, the permutation and the tile offsets are written straight
// into the caller's device buffers.  Every GPU the library runs on holds its own copy of
// the array until the process ends.  Host code never passes the array's name to a kernel
// (in host code it is only a stand-in for the symbol): the device address of each GPU's
// copy is looked up once per device with hipGetSymbolAddress and used from then on.
#include <mutex>

#include "host.h"

namespace mot {

// Largest point count of one call, and the scratch it needs: npad = max(1024, the next
// power of two >= npts) sort keys of 8 bytes, then npts tile ids of 4 bytes.
constexpr int64_t kNoAllocMaxPoints = (int64_t)1 << 20;
constexpr size_t kNoAllocKeyBytes = (size_t)kNoAllocMaxPoints * sizeof(uint64_t);
constexpr size_t kNoAllocScratchBytes = kNoAllocKeyBytes + (size_t)kNoAllocMaxPoints * sizeof(int32_t);

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;

// Device address of this GPU's scratch array, looked up on first use per device.
static int scratch_of_device(unsigned char **out)
{
    static std::mutex mu;
    static unsigned char *addr[kMaxDevices] = {};
    int dev = 0;
    MOT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return MOT_EDEVICE;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        MOT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return MOT_EDEVICE;
        addr[dev] = (unsigned char *)p;
    }
    *out = addr[dev];
    return MOT_OK;
}

}  // namespace mot

using namespace mot;

extern "C" int mot_bin_points_noalloc(int32_t d, int64_t npts, const double *x, const double *s,
                                      const double *o, int32_t n, int32_t T, int32_t sub_dim, int32_t *cell,
                                      int32_t *perm, int32_t *tile_off, void *stream)
{
    if (d < 1 || d > 3 || npts < 0 || !x || !s || !o || n < 1 || T < 1 || !cell || !perm || !tile_off)
        return MOT_EINVAL;
    if (sub_dim < -1 || sub_dim >= d || (sub_dim >= 0 && T > 16)) return MOT_EINVAL;
    const int tpd = (n + T - 1) / T;
    int64_t ntiles = 1;
    for (int c = 0; c < d; ++c) ntiles *= tpd;
    if (ntiles > ((int64_t)1 << 30) || (sub_dim >= 0 && ntiles >= ((int64_t)1 << 28))) return MOT_EINVAL;
    if (npts > kNoAllocMaxPoints) return MOT_ELIMIT;
    const size_t key_bytes = stable_tile_sort_scratch(npts, ntiles);
    if (key_bytes > kNoAllocKeyBytes) return MOT_ELIMIT;
    unsigned char *base = nullptr;
    MOT_TRY(scratch_of_device(&base));
    void *keys = base;
    int32_t *tile = (int32_t *)(base + kNoAllocKeyBytes);
    hipStream_t st = (hipStream_t)stream;
    MOT_HIP(launch_bin_cells(d, npts, x, s[0], d > 1 ? s[1] : 0.0, d > 2 ? s[2] : 0.0, o[0], d > 1 ? o[1] : 0.0,
                             d > 2 ? o[2] : 0.0, n, T, cell, tile, st));
    MOT_HIP(stable_tile_sort(npts, tile, ntiles, perm, tile_off, keys, key_bytes, st,
                             sub_dim >= 0 ? cell : nullptr, d, sub_dim >= 0 ? sub_dim : 0, T));
    return MOT_OK;
}
