// Library-owned scratch of sbp_residual_noalloc: a file-scope device array that replaces the
// caller's workspace (viscous face traces, plane-pass scratch) and the device tables the other entry
// points allocate (the collocation derivatives and the problem-group tables).
//
// In host code `scratch` names a host-side stand-in, not the device allocation: its device address
// is taken once per device with hipGetSymbolAddress (with that device current) and only that
// address is handed to kernels.
#include <mutex>

#include "sbp_internal.h"

namespace sbp {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

// Copies `n` 8-byte words carried in the kernel arguments to dst: uploads small tables without a
// host staging buffer whose lifetime would have to outlast the asynchronous call.
struct FillBlock {
    unsigned long long w[kFillWords];
};

__global__ void __launch_bounds__(256) k_fill_words(unsigned long long *dst, const FillBlock blk, int n) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = blk.w[i];
}

constexpr int kMaxDevices = 64;

}  // namespace

int fill_words(void *dst, const unsigned long long *src, long long n, hipStream_t s) {
    unsigned long long *d = static_cast<unsigned long long *>(dst);
    for (long long base = 0; base < n; base += kFillWords) {
        FillBlock blk;
        const int m = (int)((n - base) < kFillWords ? (n - base) : kFillWords);
        for (int i = 0; i < m; ++i) blk.w[i] = src[base + i];
        hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(kFillWords), 0, s, d + base, blk, m);
        if (hipGetLastError() != hipSuccess) return -1;
    }
    return 0;
}

int noalloc_scratch(const double *d_tables, long long n_words, hipStream_t s, char **ptr) {
    static std::mutex mu;
    static char *addr[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -1;
    std::lock_guard<std::mutex> lk(mu);
    if (addr[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return -1;
        // the derivative tables sit at the start of the array for the life of the process
        if (fill_words(p, reinterpret_cast<const unsigned long long *>(d_tables), n_words, s) != 0)
            return -1;
        if (hipStreamSynchronize(s) != hipSuccess) return -1;
        addr[dev] = static_cast<char *>(p);
    }
    *ptr = addr[dev];
    return 0;
}

}  // namespace sbp
