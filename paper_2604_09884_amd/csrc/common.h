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

// ------------------------------------------------------ device workspace
// Every device buffer of a handle is carved, in creation order and 256-byte
// aligned, out of one workspace: the caller's (a torch tensor, say) or, if
// the caller passes none, one allocation the handle makes and frees.  A
// sizing arena only counts bytes: running a handle's build code against it
// gives the exact workspace size without touching the device, and the same
// code then carves the real workspace.  Uploads and fills are enqueued on
// the creating stream; the host copies they read stay alive in the arena.
struct Arena {
    bool sizing = true;
    char *base = nullptr;
    size_t cap = 0, used = 0;
    hipStream_t stream = nullptr;
    std::vector<std::vector<char>> staged;
    static constexpr size_t kAlign = 256;

    void *carve(size_t n) {
        const size_t off = (used + kAlign - 1) / kAlign * kAlign;
        used = off + n;
        if (sizing || n == 0) return nullptr;
        if (used > cap) {
            set_error("workspace too small: needs more than %zu bytes", cap);
            throw Error{INRCT_EINVAL};
        }
        return base + off;
    }
};

// A buffer inside a handle's workspace (not owned separately).
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    void alloc(Arena &a, size_t n) {
        ptr = a.carve(n);
        bytes = n;
    }
    template <class T> T *as() const { return reinterpret_cast<T *>(ptr); }
};

// Fills `n` bytes with zero using a kernel (capturable; no memset node).
void launch_zero_bytes(void *p, size_t n, hipStream_t s);

template <class T>
void upload(Arena &a, DevBuf &b, const std::vector<T> &v) {
    const size_t n = v.size() * sizeof(T);
    b.alloc(a, n);
    if (a.sizing || n == 0) return;
    a.staged.emplace_back((const char *)v.data(), (const char *)v.data() + n);
    INRCT_CHECK_HIP(hipMemcpyAsync(b.ptr, a.staged.back().data(), n, hipMemcpyHostToDevice,
                                   a.stream));
}

inline void zero_fill(Arena &a, DevBuf &b) {
    if (!a.sizing) launch_zero_bytes(b.ptr, b.bytes, a.stream);
}

// The workspace of a handle: the arena it was carved with and, when the
// library allocated it, that allocation.
struct Workspace {
    Arena arena;
    void *owned = nullptr;
    ~Workspace() {
        if (owned) (void)hipFree(owned);
    }
};

// Builds a handle in two passes: `build(arena)` against a sizing arena (on a
// scratch copy of the handle, made by `fresh`) to learn the workspace size,
// then against the real workspace -- `ws` if given (at least that large and
// 256-byte aligned), else one hipMalloc owned by the handle.
template <class H, class Fresh, class Build>
void build_in_workspace(H *h, Workspace &w, void *ws, size_t ws_bytes, hipStream_t s,
                        Fresh &&fresh, Build &&build) {
    size_t need = 0;
    {
        H *tmp = fresh();
        Arena sz;
        try {
            build(tmp, sz);
        } catch (...) {
            delete tmp;
            throw;
        }
        delete tmp;
        need = sz.used;
    }
    Arena &a = w.arena;
    a.sizing = false;
    a.stream = s;
    if (ws) {
        if (ws_bytes < need) {
            set_error("workspace of %zu bytes is too small: this handle needs %zu "
                      "(inrct_workspace_bytes)", ws_bytes, need);
            throw Error{INRCT_EINVAL};
        }
        if ((uintptr_t)ws % Arena::kAlign) {
            set_error("workspace must be %zu-byte aligned", Arena::kAlign);
            throw Error{INRCT_EINVAL};
        }
        a.base = (char *)ws;
        a.cap = ws_bytes;
    } else if (need > 0) {
        hipError_t e = hipMalloc(&w.owned, need);
        if (e != hipSuccess) {
            w.owned = nullptr;
            set_error("hipMalloc(%zu) failed: %s", need, hipGetErrorString(e));
            throw Error{INRCT_ENOMEM};
        }
        a.base = (char *)w.owned;
        a.cap = need;
    }
    build(h, a);
}

// Runs only the sizing pass: the workspace bytes a handle built by `build`
// needs.
template <class H, class Fresh, class Build>
size_t workspace_need(Fresh &&fresh, Build &&build) {
    H *tmp = fresh();
    Arena sz;
    try {
        build(tmp, sz);
    } catch (...) {
        delete tmp;
        throw;
    }
    delete tmp;
    return sz.used;
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
    void build(Arena &a, int dim, int N);
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
}  // namespace inrct
