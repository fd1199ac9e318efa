// Error reporting, FOV tables and small utility kernels.
#include <stdarg.h>

#include "common.h"

namespace inrct {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

const char *last_error() { return g_last_error.c_str(); }

void FovHost::build(Arena &ar, int dim, int N) {
    xlo.assign(N, 0);
    cnt.assign(N, 0);
    row_start.assign(N + 1, 0);
    // centre c(i) = (2i + 1 - N)/N; c(x)^2 + c(y)^2 <= 1 in exact integers
    const int64_t NN = (int64_t)N * N;
    int64_t acc = 0;
    for (int y = 0; y < N; ++y) {
        int64_t a = 2LL * y + 1 - N;
        int first = -1, last = -2;
        for (int x = 0; x < N; ++x) {
            int64_t b = 2LL * x + 1 - N;
            if (a * a + b * b <= NN) {
                if (first < 0) first = x;
                last = x;
            }
        }
        row_start[y] = (int32_t)acc;
        if (first >= 0) {
            xlo[y] = first;
            cnt[y] = last - first + 1;
        }
        acc += cnt[y];
    }
    row_start[N] = (int32_t)acc;
    n_slice = acc;
    n = acc * (dim == 3 ? N : 1);
    upload(ar, d_xlo, xlo);
    upload(ar, d_row_start, row_start);
}

__global__ void k_sum_partials(const double *p, int n, double *out) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += p[i];
    double s = block_sum_f64(acc, sh);
    if (threadIdx.x == 0) *out = s;
}

void launch_sum_partials(const double *partials, int n, double *out,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, n,
                       out);
    INRCT_CHECK_LAUNCH();
}

__global__ void k_zero16(uint4 *p, size_t n16) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_zero1(unsigned char *p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

void launch_zero_bytes(void *p, size_t n, hipStream_t s) {
    if (n == 0) return;
    size_t head = 0;
    uintptr_t a = (uintptr_t)p;
    if (a % 16) head = 16 - a % 16;
    if (head > n) head = n;
    if (head) {
        hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, s, (unsigned char *)p,
                           head);
        INRCT_CHECK_LAUNCH();
    }
    size_t body = (n - head) / 16;
    if (body) {
        size_t blocks = (size_t)cdiv((int64_t)body, 256);
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_zero16, dim3((unsigned)blocks), dim3(256), 0, s,
                           (uint4 *)((char *)p + head), body);
        INRCT_CHECK_LAUNCH();
    }
    size_t tail = n - head - body * 16;
    if (tail) {
        hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, s,
                           (unsigned char *)p + head + body * 16, tail);
        INRCT_CHECK_LAUNCH();
    }
}

}  // namespace inrct

extern "C" const char *inrct_last_error(void) { return inrct::last_error(); }
