// lh_noalloc.hip -- the q-average of output planes with a device-resident
// scratch array instead of plan memory: for callers that cannot allocate
// device memory (code under stream capture, serving loops, harnesses that
// forbid it).  No hipMalloc, hipFree or allocating library call on this path.
#include <mutex>
#include <vector>

#include "lh_internal.h"

namespace lh {

// Partial sums of the q-average: kQavgBlocks doubles per plane, at most
// LINDHARD_NOALLOC_MAX_PLANES planes (1 MiB).  Each device holds its own copy
// for the life of the process.  Every entry a call reads was written by that
// call's first kernel, so nothing needs clearing; calls that overlap on one
// device race on it.
static __device__ __align__(256) double scratch[(size_t)LINDHARD_NOALLOC_MAX_PLANES * kQavgBlocks];

namespace {
std::mutex g_scratch_mu;
std::vector<double *> g_scratch_ptr;  // device address of `scratch` per device (null until set up)

// Device address of this device's scratch array, looked up once per device
// with that device current.  nullptr on failure.
double *scratch_ptr(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((size_t)device >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    return g_scratch_ptr[device];
}
}  // namespace

}  // namespace lh

using namespace lh;

extern "C" lindhard_status lindhard_q_average_noalloc(const void *im, int32_t nomega, int64_t plane_elems,
                                                      int32_t elem_bytes, double *out, void *stream)
{
    if (!im || !out || plane_elems < 1 || (elem_bytes != 4 && elem_bytes != 8)) return LINDHARD_EINVAL;
    if (nomega < 1 || nomega > LINDHARD_NOALLOC_MAX_PLANES) return LINDHARD_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINDHARD_EDEVICE;
    double *part = scratch_ptr(dev);
    if (!part) return LINDHARD_EDEVICE;
    const hipError_t e = launch_qavg_raw(im, elem_bytes == 8, (size_t)plane_elems, nomega, part, out,
                                         (hipStream_t)stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return LINDHARD_EDEVICE;
    }
    return LINDHARD_OK;
}
