// ebr_score_topk_noalloc: the top-K batch of ebr_score_topk with its workspace in a fixed
// device array of this library instead of a caller buffer, for callers that cannot allocate
// (code under stream capture, serving loops that forbid allocation).
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "internal.h"

namespace ebr {

// The array: one per GPU the library runs on, held until the process ends. Host code never
// passes its name to a kernel (on the host it is a stand-in, not a device address); it uses
// the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[EBR_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on device `dev` (the current device), looked up once per device.
static ebr_status scratch_address(int dev, char** out) {
    static std::mutex mu;
    static std::vector<char*> addr;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)addr.size() <= dev) addr.resize((size_t)dev + 1, nullptr);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return EBR_EDEVICE;
        }
        addr[dev] = (char*)p;
    }
    *out = addr[dev];
    return EBR_OK;
}

}  // namespace ebr

extern "C" ebr_status ebr_score_topk_noalloc(const ebr_index* index, const ebr_batch* batch,
                                             uint32_t* out_ids, float* out_scores, void* hip_stream) {
    using namespace ebr;
    try {
        if (!index) { set_error("index is NULL"); return EBR_EINVAL; }
        size_t need = 0;
        ebr_status st = ebr_workspace_size(index, batch, &need);
        if (st) return st;
        if (need > (size_t)EBR_NOALLOC_SCRATCH_BYTES) {
            set_error("batch needs %zu bytes of workspace, more than the %zu-byte static scratch of "
                      "ebr_score_topk_noalloc (use ebr_score_topk with a caller workspace)",
                      need, (size_t)EBR_NOALLOC_SCRATCH_BYTES);
            return EBR_ENOMEM;
        }
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) { set_error("hipGetDevice failed"); return EBR_EDEVICE; }
        char* ws = nullptr;
        st = scratch_address(dev, &ws);
        if (st) return st;
        return run_topk(*index, batch, ws, (size_t)EBR_NOALLOC_SCRATCH_BYTES, out_ids, out_scores,
                        hip_stream, nullptr);
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    }
}
