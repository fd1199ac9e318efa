// Internal helpers shared by the HIP sources of libinrct (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string>
#include <vector>

#include "inrct.h"

namespace inrct {

// ----------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
void clear_error();

struct Error {
    int code;
};

#define INRCT_CHECK_HIP(expr)                                                  \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            ::inrct::set_error("%s failed: %s (%s:%d)", #expr,                 \
                               hipGetErrorString(e_), __FILE__, __LINE__);     \
            throw ::inrct::Error{INRCT_EHIP};                                  \
        }                                                                      \
    } while (0)

#define INRCT_CHECK_LAUNCH() INRCT_CHECK_HIP(hipGetLastError())

#define INRCT_REQUIRE(cond, ...)                                               \
    do {                                                                       \
        if (!(cond)) {                                                         \
            ::inrct::set_error(__VA_ARGS__);                                   \
            throw ::inrct::Error{INRCT_EINVAL};                                \
        }                                                                      \
    } while (0)

// Runs `body` and converts thrown errors to status codes.
template <class F>
int guarded(F &&body) {
    clear_error();
    try {
        body();
        return INRCT_OK;
    } catch (const Error &e) {
        return e.code;
    } catch (...) {
        set_error("unexpected C++ exception");
        return INRCT_EINVAL;
    }
}

// Device buffer owned by a handle; freed with the handle.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    void alloc(size_t n) {
        release();
        if (n == 0) return;
        hipError_t e = hipMalloc(&ptr, n);
        if (e != hipSuccess) {
            ptr = nullptr;
            set_error("hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
            throw Error{INRCT_ENOMEM};
        }
        bytes = n;
    }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return reinterpret_cast<T *>(ptr); }
    ~DevBuf() { release(); }
};

template <class T>
void upload(DevBuf &b, const std::vector<T> &v) {
    b.alloc(v.size() * sizeof(T));
    if (!v.empty())
        INRCT_CHECK_HIP(hipMemcpy(b.ptr, v.data(), v.size() * sizeof(T),
                                  hipMemcpyHostToDevice));
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------- FOV tables
// The FOV of one z-slice is a disc; row y holds the contiguous x range
// [xlo[y], xlo[y] + cnt[y]).  row_start[y] is the rank of the row's first
// point within the slice; n_slice the slice total.  Rank q of the whole
// FOV: z = q / n_slice, then y by binary search over row_start.
struct FovDev {
    const int32_t *xlo;
    const int32_t *row_start;  // [N + 1]
    int32_t n_slice;
    int32_t N;
    int32_t dim;
};

struct FovHost {
    std::vector<int32_t> xlo, cnt, row_start;
    int64_t n_slice = 0, n = 0;
    DevBuf d_xlo, d_row_start;
    void build(int dim, int N);
    FovDev dev(int dim) const {
        return FovDev{d_xlo.as<int32_t>(), d_row_start.as<int32_t>(),
                      (int32_t)n_slice, (int32_t)xlo.size(), dim};
    }
};

__device__ __forceinline__ int64_t fov_rank_to_index(const FovDev &f,
                                                     int64_t q, int *ox,
                                                     int *oy, int *oz) {
    int z = (int)(q / f.n_slice);
    int rem = (int)(q - (int64_t)z * f.n_slice);
    int lo = 0, hi = f.N;  // find last y with row_start[y] <= rem
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (f.row_start[mid] <= rem) lo = mid; else hi = mid;
    }
    int y = lo;
    int x = f.xlo[y] + (rem - f.row_start[y]);
    *ox = x;
    *oy = y;
    *oz = z;
    return ((int64_t)z * f.N + y) * f.N + x;
}

// ------------------------------------------------------- fixed-order sums
// Block-level float64 sum of one value per thread (blockDim.x == 256).
__device__ __forceinline__ double block_sum_f64(double v, double *sh) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Reduces `n` float64 partials in a fixed order into *out (one block).
void launch_sum_partials(const double *partials, int n, double *out,
                         hipStream_t s);
// Fills `n` bytes with zero using a kernel (capturable; no memset node).
void launch_zero_bytes(void *p, size_t n, hipStream_t s);

}  // namespace inrct
