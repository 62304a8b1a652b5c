// fewha_dwt_forward_noalloc: the forward transform W with its scratch in a library-owned device
// array instead of the plan workspace, for callers that cannot allocate device memory.
//
// The levels past the fine tiles (kf + 1 .. J) start from the level-kf approximation of every
// layer, which the fine-level launch leaves in scratch memory.  fewha_dwt_forward takes that
// scratch from the bound workspace; this entry point takes it from `scratch` below, so it runs on
// a created plan whether or not a workspace was ever bound.  The array lives in every GPU's
// memory from the library's load until the process ends; its address on a device is looked up
// once, with that device current, and kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

using namespace fewha;

namespace {

// Largest scratch a call may need: the level-kf approximation of every layer (at most
// n_coef / 4 + 4 values), 8 MiB: up to 8.3 M coefficients in FP32, 4.1 M in FP64.
constexpr size_t kScratchBytes = size_t(8) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device set up so far

// The address of `scratch` on the current device (first use on a device: look it up and set the
// kernels' dynamic LDS limits there).  The array's host-side name is only a stand-in, so kernels
// and copies get this address, never `scratch` itself.
template <typename T>
int device_scratch(const Plan &P, void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return FEWHA_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return FEWHA_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_failure(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        Ops<T> o{P, Bufs<T>{}, nullptr};
        if (int st = o.prepare()) return st;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return FEWHA_OK;
}

template <typename T>
int forward(const Plan &P, const void *layers, void *c, void *stream) {
    const size_t need = P.kf < P.J ? ll_stride(P.n_coef) * sizeof(T) : 0;
    if (need > kScratchBytes) return FEWHA_ERR_UNSUPPORTED;
    void *ptr = nullptr;
    if (int st = device_scratch<T>(P, &ptr)) return st;
    Bufs<T> B{};  // the transform reads only its input and the approximation scratch
    B.ll = static_cast<T *>(ptr);
    B.fs_c = (long)P.n_coef;
    B.fs_v = (long)P.n_nodes;
    B.fs_s = (long)P.n_slopes;
    B.fs_a = (long)P.n_act;
    B.fs_ll = (long)ll_stride(P.n_coef);
    Ops<T> o{P, B, static_cast<hipStream_t>(stream)};
    FwdArgs E{};
    E.out = c;
    return o.fwd(static_cast<const T *>(layers), E, kEpiPlain);
}

}  // namespace

extern "C" int fewha_dwt_forward_noalloc(const fewha_plan *p, const void *d_layers, void *d_c, void *stream) {
    if (!p || !d_layers || !d_c || d_layers == d_c) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? forward<double>(p->p, d_layers, d_c, stream)
                                   : forward<float>(p->p, d_layers, d_c, stream);
}
