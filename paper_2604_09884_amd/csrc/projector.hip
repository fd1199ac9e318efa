// 2D parallel- and fan-beam Joseph projector P, its voxel-driven exact
// transpose P^T, the data-fidelity residuals (Sec. II, Sec. III of the
// paper) and the geometry handle.  The cone-beam kernels are in cone.hip.
//
// Geometry is reduced on the host, in float64, to one record per (view,
// detector bin): the interpolation position of the ray's non-principal
// coordinate as a 32.32 fixed-point start value and per-slice increment,
// and the slice step length.  Because the interpolation position at slice
// s is the exact integer F0 + s * dF in both kernels, P^T applies exactly
// the weights P applies.
#include <math.h>

#include "geom.h"

namespace inrct {

static const double kFix = 4294967296.0;       // 2^32
static const float kInvFix = 2.3283064365386963e-10f;  // 2^-32

// ------------------------------------------------------------- host tables
// Per (view, bin) ray geometry in float64, before it is reduced to the
// device tables.
struct RayGeom {
    long long F0, dF;  // 32.32 fixed point phi_other at slice 0, per slice
    double step;       // h |d| / |d_axis|
    int ypr;           // 1: y is the principal axis
};

static void build_tables(const ct_geometry &g, int N, std::vector<Col2D> &cols,
                         std::vector<float> &steps, std::vector<View2D> &views) {
    const double h = 2.0 / N;
    const double c0 = -1.0 + 0.5 * h;
    const double tau = 1e-9;
    const bool fan = g.kind != INRCT_PAR2D;
    cols.resize((size_t)g.n_views * g.n_u);
    steps.resize(cols.size());
    views.resize(g.n_views);
    std::vector<RayGeom> rg(g.n_u);
    for (int j = 0; j < g.n_views; ++j) {
        const double th = g.angles[j];
        const double cs = cos(th), sn = sin(th);
        // fan: source S, detector centre C, detector axis e_u (the in-plane
        // part of the cone geometry); parallel: rays (-sin, cos) through
        // u (cos, sin)
        const double Sx = g.sid * cs, Sy = g.sid * sn, Cx = -g.idd * cs, Cy = -g.idd * sn;
        const double eux = fan ? -sn : cs, euy = fan ? cs : sn;
        for (int a = 0; a < g.n_u; ++a) {
            const double ua = ((double)a - 0.5 * (double)(g.n_u - 1)) * g.du;
            double p0x, p0y, dx, dy;
            if (fan) {
                p0x = Sx;
                p0y = Sy;
                dx = Cx - Sx + ua * eux;
                dy = Cy - Sy + ua * euy;
            } else {
                p0x = ua * cs;
                p0y = ua * sn;
                dx = -sn;
                dy = cs;
            }
            RayGeom &r = rg[a];
            r.ypr = fabs(dy) >= (1.0 - tau) * fabs(dx) ? 1 : 0;
            const double dax = r.ypr ? dy : dx;
            const double dot = r.ypr ? dx : dy;
            const double pax = r.ypr ? p0y : p0x;
            const double pot = r.ypr ? p0x : p0y;
            const double inv = 1.0 / dax;
            const double t0 = (c0 - pax) * inv;
            const double phi0 = (pot + t0 * dot + 1.0) / h - 0.5;
            r.F0 = llrint(phi0 * kFix);
            r.dF = llrint(dot * inv * kFix);
            r.step = h * sqrt(dx * dx + dy * dy) * fabs(inv);
        }
        int changes = 0, split = g.n_u;
        for (int a = 1; a < g.n_u; ++a)
            if (rg[a].ypr != rg[a - 1].ypr) {
                ++changes;
                split = a;
            }
        if (changes > 1) {
            set_error("view %d: the fan crosses two principal-axis boundaries (wider than 90 "
                      "degrees)", j);
            throw Error{INRCT_EINVAL};
        }
        View2D &vg = views[j];
        vg.sx = (float)(fan ? Sx : 0.0);
        vg.sy = (float)(fan ? Sy : 0.0);
        vg.ax = (float)(fan ? Sx - Cx : 0.0);
        vg.ay = (float)(fan ? Sy - Cy : 0.0);
        vg.eux = (float)eux;
        vg.euy = (float)euy;
        vg.ysplit = split;
        vg.yfirst = rg[0].ypr;
        for (int a = 0; a < g.n_u; ++a) {
            cols[(size_t)j * g.n_u + a] = Col2D{rg[a].F0, rg[a].dF};
            steps[(size_t)j * g.n_u + a] = (float)rg[a].step;
        }
    }
}

// --------------------------------------------------------- device helpers
__device__ __forceinline__ int fx_int(long long F) { return (int)(F >> 32); }
__device__ __forceinline__ float fx_frac(long long F) {
    return (float)(unsigned int)(F & 0xffffffffLL) * kInvFix;
}
__device__ __forceinline__ bool bin_ypr(const View2D &vg, int a) {
    return (a < vg.ysplit) == (vg.yfirst != 0);
}

// Slices s in [0, N) whose interpolation index floor(phi(s)) can touch the
// grid, i.e. -1 <= phi(s) < N (a superset: taps are bounds-checked anyway).
__device__ __forceinline__ void slice_range(long long F0, long long dF, int N,
                                            int *lo, int *hi) {
    const double phi0 = (double)F0 * (1.0 / kFix);
    const double sl = (double)dF * (1.0 / kFix);
    double a, b;
    if (sl > 0) {
        a = (-1.0 - phi0) / sl;
        b = ((double)N - phi0) / sl;
    } else if (sl < 0) {
        a = ((double)N - phi0) / sl;
        b = (-1.0 - phi0) / sl;
    } else {
        if (phi0 >= -1.0 && phi0 < (double)N) { a = 0; b = N - 1; }
        else { a = 1; b = 0; }
    }
    double l = floor(a) - 1.0, r = ceil(b) + 1.0;
    if (l < 0) l = 0;
    if (r > N - 1) r = N - 1;
    *lo = (int)l;
    *hi = (int)r;
}

// ----------------------------------------------------------- forward, 2D
// ut = u transposed in every xy plane ([z][x][y]; blockIdx.z is the plane),
// so that x-principal rays read rows too.
__global__ __launch_bounds__(256) void k_transpose2d(const float *__restrict__ u,
                                                     float *__restrict__ ut, int N) {
    __shared__ float t[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    u += (size_t)blockIdx.z * N * N;
    ut += (size_t)blockIdx.z * N * N;
    for (int k = 0; k < 32; k += 8) {
        const int x = x0 + tx, y = y0 + ty + k;
        if (x < N && y < N) t[ty + k][tx] = u[(size_t)y * N + x];
    }
    __syncthreads();
    for (int k = 0; k < 32; k += 8) {
        const int y = y0 + tx, x = x0 + ty + k;
        if (x < N && y < N) ut[(size_t)x * N + y] = t[tx][ty + k];
    }
}

// A workgroup covers 64 consecutive bins of one view (one bin per lane);
// its four waves integrate four consecutive quarters of every ray's slice
// range, and the quarters are added in order.  At slice s a y-principal ray
// reads row s of u, an x-principal ray row s of ut, so neighbouring bins
// read neighbouring addresses either way.
__global__ __launch_bounds__(256) void k_proj2d(GeomDev g, const float *__restrict__ u,
                                                const float *__restrict__ ut,
                                                float *__restrict__ z) {
    __shared__ float part[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int a = blockIdx.x * 64 + lane;
    const int j = blockIdx.y;
    const int N = g.N;
    float acc = 0.f;
    if (a < g.Nu) {
        const Col2D c = g.col[(size_t)j * g.Nu + a];
        const float *src = bin_ypr(g.view[j], a) ? u : ut;
        int lo, hi;
        slice_range(c.F0, c.dF, N, &lo, &hi);
        const int q = (hi - lo + 4) >> 2;  // ceil(len / 4), len = hi - lo + 1
        const int s0 = lo + w * q, s1 = min(hi, s0 + q - 1);
        long long F = c.F0 + (long long)s0 * c.dF;
        for (int s = s0; s <= s1; ++s, F += c.dF) {
            const int io = fx_int(F);
            const float wt = fx_frac(F);
            const float *row = src + (size_t)s * N;
            const float v0 = (unsigned)io < (unsigned)N ? row[io] : 0.f;
            const float v1 = (unsigned)(io + 1) < (unsigned)N ? row[io + 1] : 0.f;
            acc += (1.f - wt) * v0 + wt * v1;
        }
    }
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0 && a < g.Nu)
        z[(size_t)j * g.Nu + a] =
            (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]) *
            g.step[(size_t)j * g.Nu + a];
}

// ------------------------------------------------ adjoint (gather) helpers
// Bins whose ray crosses the in-plane segment p1-p2 (the bins at positions
// inside the segment's image on the detector), in single precision and
// widened by 0.01 bin, far above its rounding error: every candidate is
// then tested exactly on the fixed-point stencil, so an extra candidate
// costs time but never changes a sum.  Parallel beam: the segment's
// projection on the detector axis.  Fan beam: the central projection of its
// end points from the source onto the detector line (monotone along the
// segment, since the segment lies on the detector's side of the line
// through the source parallel to the detector).
template <bool FAN>
__device__ __forceinline__ void cand_bins(const GeomDev &g, const View2D &vg, float p1x,
                                          float p1y, float p2x, float p2y, float inv_du,
                                          int *lo, int *hi) {
    float u1, u2;
    if (FAN) {
        const float D1x = p1x - vg.sx, D1y = p1y - vg.sy;
        const float D2x = p2x - vg.sx, D2y = p2y - vg.sy;
        // hardware reciprocal (about 1 ulp): far inside the 0.01-bin margin
        u1 = (vg.ax * D1y - vg.ay * D1x) *
             __builtin_amdgcn_rcpf(vg.eux * D1y - vg.euy * D1x);
        u2 = (vg.ax * D2y - vg.ay * D2x) *
             __builtin_amdgcn_rcpf(vg.eux * D2y - vg.euy * D2x);
    } else {
        u1 = p1x * vg.eux + p1y * vg.euy;
        u2 = p2x * vg.eux + p2y * vg.euy;
    }
    const float c = 0.5f * (float)(g.Nu - 1);
    const float a1 = u1 * inv_du + c, a2 = u2 * inv_du + c;
    // the bins inside [a1, a2], widened by the margin
    float l = ceilf(fminf(a1, a2) - 0.01f), r = floorf(fmaxf(a1, a2) + 0.01f);
    l = fmaxf(l, 0.f);
    r = fminf(r, (float)(g.Nu - 1));
    *lo = (int)l;
    *hi = (int)r;
}

// The part of (P^T r) at pixel (ix, iy) from views [j0, j1): rs is the
// step-weighted residual r * step.  Views in order; per view the
// y-principal bins, then the x-principal ones, each in ascending order.
template <bool FAN>
__device__ float bp_pixel_2d(const GeomDev &g, const float *__restrict__ rs, int ix, int iy,
                             int j0, int j1) {
    const float h = (float)g.h;
    const float x = (float)(-1.0 + (ix + 0.5) * g.h), y = (float)(-1.0 + (iy + 0.5) * g.h);
    const float inv_du = (float)(1.0 / g.du);
    const int Nu = g.Nu;
    float acc = 0.f;
    for (int j = j0; j < j1; ++j) {
        const View2D vg = g.view[j];
        const float *rj = rs + (size_t)j * Nu;
        const Col2D *cj = g.col + (size_t)j * Nu;
        for (int pass = 0; pass < 2; ++pass) {
            const bool ypass = pass == 0;
            // the run of bins with this principal axis
            int blo = (ypass == (vg.yfirst != 0)) ? 0 : vg.ysplit;
            int bhi = (ypass == (vg.yfirst != 0)) ? vg.ysplit - 1 : Nu - 1;
            if (blo > bhi) continue;
            const int s = ypass ? iy : ix, o = ypass ? ix : iy;
            int lo, hi;
            if (ypass) cand_bins<FAN>(g, vg, x - h, y, x + h, y, inv_du, &lo, &hi);
            else cand_bins<FAN>(g, vg, x, y - h, x, y + h, inv_du, &lo, &hi);
            lo = max(lo, blo);
            hi = min(hi, bhi);
            for (int a = lo; a <= hi; ++a) {
                const Col2D c = cj[a];
                const long long F = c.F0 + (long long)s * c.dF;
                const int i0 = fx_int(F);
                const float wt = fx_frac(F);
                if (i0 == o) acc += (1.f - wt) * rj[a];
                else if (i0 == o - 1) acc += wt * rj[a];
            }
        }
    }
    return acc;
}

// rs = r * step length (applied on the ray side of P^T)
__global__ __launch_bounds__(256) void k_prescale2d(GeomDev g, const float *__restrict__ r,
                                                    float *__restrict__ rs) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < (int64_t)g.V * g.Nu) rs[i] = r[i] * g.step[i];
}

// A workgroup covers an 8 x 8 patch of pixels (one per lane); its four
// waves gather four consecutive quarters of the views, added in order.
template <bool FAN>
__global__ __launch_bounds__(256) void k_bproj2d(GeomDev g, const float *__restrict__ rs,
                                                 float *__restrict__ v) {
    __shared__ float part[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int ix = blockIdx.x * 8 + (lane & 7);
    const int iy = blockIdx.y * 8 + (lane >> 3);
    const bool in = ix < g.N && iy < g.N;
    const int q = (g.V + 3) >> 2;
    const int j0 = min(g.V, w * q), j1 = min(g.V, j0 + q);
    part[w][lane] = in ? bp_pixel_2d<FAN>(g, rs, ix, iy, j0, j1) : 0.f;
    __syncthreads();
    if (w == 0 && in)
        v[(size_t)iy * g.N + ix] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

template <bool FAN>
__global__ __launch_bounds__(256) void k_bproj_at(GeomDev g, const float *__restrict__ rs,
                                                  const int32_t *__restrict__ idx,
                                                  int64_t k, float *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= k) return;
    const int64_t q = idx[t];
    const int N = g.N;
    const int ix = (int)(q % N), iy = (int)((q / N) % N);
    // the same view quarters, added in the same order, as k_bproj2d
    const int qv = (g.V + 3) >> 2;
    float acc = 0.f;
    for (int w = 0; w < 4; ++w) {
        const int j0 = min(g.V, w * qv), j1 = min(g.V, j0 + qv);
        const float p = bp_pixel_2d<FAN>(g, rs, ix, iy, j0, j1);
        acc = w == 0 ? p : acc + p;
    }
    out[t] = acc;
}

// ---------------------------------------------------------------- residual
__global__ __launch_bounds__(256) void k_residual_ls(const float *__restrict__ z,
                                                     const float *__restrict__ y,
                                                     float *r, int64_t m,
                                                     double *partials) {
    __shared__ double sh[256];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += stride) {
        const float d = z[i] - y[i];
        r[i] = d;
        acc += (double)d * (double)d;
    }
    const double s = block_sum_f64(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = 0.5 * s;
}

__global__ __launch_bounds__(256) void k_diff(const float *__restrict__ z,
                                              const float *__restrict__ y,
                                              float *__restrict__ q, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) q[i] = z[i] - y[i];
}

// r = F q along each detector row (Ram-Lak, linear convolution), and the
// per-block partials of 1/2 q.r.  Row length nu, rows = m / nu.  A block
// takes rows blockIdx.x, blockIdx.x + gridDim.x, ...: the row is staged in
// LDS between nu zeros on each side (so no tap needs a bounds test) and the
// odd taps f_j = -1 / (pi^2 j^2 du) are computed once per block; each
// output sums its taps in increasing j.  LDS: 3 nu + nu / 2 floats.
__global__ __launch_bounds__(256) void k_ramp(const float *__restrict__ q, float *r, int nu,
                                              int64_t rows, double du, double *partials) {
    extern __shared__ float lds[];
    float *row = lds;               // [3 nu]: zeros, the row, zeros
    float *tap = lds + 3 * nu;      // [nu / 2]: f_{2i+1}
    __shared__ double sh[256];
    const float f0 = (float)(1.0 / (4.0 * du));
    const float cf = (float)(-1.0 / (M_PI * M_PI * du));
    const int nt = nu / 2;          // odd offsets 1, 3, ..., < nu
    for (int i = threadIdx.x; i < nt; i += 256) {
        const int jj = 2 * i + 1;
        tap[i] = cf / ((float)jj * (float)jj);
    }
    for (int i = threadIdx.x; i < nu; i += 256) {
        row[i] = 0.f;
        row[2 * nu + i] = 0.f;
    }
    double acc = 0.0;
    for (int64_t rw = blockIdx.x; rw < rows; rw += gridDim.x) {
        const float *qr = q + rw * nu;
        __syncthreads();  // the previous row's reads are done
        for (int i = threadIdx.x; i < nu; i += 256) row[nu + i] = qr[i];
        __syncthreads();
        for (int a = threadIdx.x; a < nu; a += 256) {
            const float *c = row + nu + a;
            float s = f0 * c[0];
            for (int i = 0; i < nt; ++i) {
                const int jj = 2 * i + 1;
                s += tap[i] * (c[-jj] + c[jj]);
            }
            r[rw * nu + a] = s;
            acc += 0.5 * (double)c[0] * (double)s;
        }
    }
    const double tot = block_sum_f64(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// The same filter, register-tiled: a thread computes B consecutive outputs
// a0 .. a0 + B - 1 of a row (B odd, so the lanes' LDS addresses, B words
// apart, fall in distinct banks).  At odd offset j the outputs need the inputs
// at a - j and a + j: two windows of B values, which move by two values at
// the next odd offset.  The windows are circular register buffers whose
// rotation is fixed at compile time (B taps per unrolled group), so a tap
// reads four new values from LDS for 2B operations instead of three for two.
// Each output adds its terms in k_ramp's order (the same float result).  A
// workgroup holds `rpb` rows at once, `tpr` threads each.
constexpr int kRampPad = 16;  // zero floats before and after a staged row (>= B)

template <int B>
__global__ __launch_bounds__(256) void k_ramp_tiled(const float *__restrict__ q,
                                                    float *__restrict__ r, int nu, int64_t rows,
                                                    int tpr, int rpb, double du,
                                                    double *__restrict__ partials) {
    extern __shared__ float lds[];
    const int nt = nu / 2;  // odd offsets 1, 3, ..., < nu
    const int stride = 3 * nu + 2 * kRampPad;
    float *tap = lds;                // [nt]: f_{2i+1}
    float *rowbuf = lds + nt;        // rpb x [pad, nu zeros, the row, nu zeros, pad]
    __shared__ double sh[256];
    const float f0 = (float)(1.0 / (4.0 * du));
    const float cf = (float)(-1.0 / (M_PI * M_PI * du));
    for (int i = threadIdx.x; i < nt; i += 256) {
        const int jj = 2 * i + 1;
        tap[i] = cf / ((float)jj * (float)jj);
    }
    for (int i = threadIdx.x; i < rpb * stride; i += 256) rowbuf[i] = 0.f;
    const int grp = threadIdx.x / tpr, t = threadIdx.x - grp * tpr;
    const int a0 = t * B;
    const bool mine = grp < rpb;
    const float *c = rowbuf + (mine ? grp : 0) * stride + kRampPad + nu;  // c[0]: the row's first value
    double acc = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * rpb; base < rows;
         base += (int64_t)gridDim.x * rpb) {
        const int64_t rw = base + grp;
        const bool live = mine && rw < rows;
        __syncthreads();  // the previous rows' reads are done
        if (live) {
            float *dst = rowbuf + grp * stride + kRampPad + nu;
            for (int i = t; i < nu; i += tpr) dst[i] = q[rw * nu + i];
        }
        __syncthreads();
        if (!live || a0 >= nu) continue;
        float sum[B], L[B], R[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            sum[b] = f0 * c[a0 + b];
            L[b] = c[a0 + b - 1];
            R[b] = c[a0 + b + 1];
        }
        // at step u of a group, L[b] (the input at a0 + b - j) sits in slot
        // (b - 2u) mod B and R[b] (at a0 + b + j) in slot (b + 2u) mod B
        for (int i0 = 0; i0 < nt; i0 += B) {
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int i = i0 + u;
                if (i < nt) {
                    const int jj = 2 * i + 1;
                    const float tp = tap[i];
#pragma unroll
                    for (int b = 0; b < B; ++b)
                        sum[b] += tp * (L[((b - 2 * u) % B + B) % B] + R[(b + 2 * u) % B]);
                    // the next offset's new values: L[0], L[1] and R[B-2], R[B-1]
                    L[((-2 * (u + 1)) % B + B) % B] = c[a0 - jj - 2];
                    L[((1 - 2 * (u + 1)) % B + B) % B] = c[a0 - jj - 1];
                    R[(2 * u) % B] = c[a0 + B + jj];
                    R[(2 * u + 1) % B] = c[a0 + B + 1 + jj];
                }
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b)
            if (a0 + b < nu) {
                r[rw * nu + a0 + b] = sum[b];
                acc += 0.5 * (double)c[a0 + b] * (double)sum[b];
            }
    }
    const double tot = block_sum_f64(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

}  // namespace inrct

// ==================================================================== ABI
using namespace inrct;

namespace inrct {
int64_t geom_rays(const inrct_geom *g) { return g->m(); }
int geom_dim(const inrct_geom *g) { return g->dim; }
int geom_N(const inrct_geom *g) { return g->N; }

void transpose_planes(const float *u, float *ut, int N, int planes, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose2d, dim3((unsigned)cdiv(N, 32), (unsigned)cdiv(N, 32), planes),
                       dim3(256), 0, s, u, ut, N);
    INRCT_CHECK_LAUNCH();
}

void project(inrct_geom *geom, const float *u, float *z, hipStream_t s, bool fov_only,
             const float *ut) {
    const GeomDev d = geom->dev();
    if (d.kind == INRCT_PAR2D || d.kind == INRCT_FAN2D) {
        float *ut = geom->ut.as<float>();
        hipLaunchKernelGGL(k_transpose2d, dim3((unsigned)cdiv(d.N, 32), (unsigned)cdiv(d.N, 32)),
                           dim3(256), 0, s, u, ut, d.N);
        INRCT_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_proj2d, dim3((unsigned)cdiv(d.Nu, 64), d.V), dim3(256),
                           0, s, d, u, ut, z);
        INRCT_CHECK_LAUNCH();
    } else {
        cone_project(geom, u, z, fov_only, s, ut);
    }
}

static const float *prescale2d(inrct_geom *geom, const float *r, hipStream_t s) {
    const GeomDev d = geom->dev();
    float *rs = geom->q.as<float>();
    hipLaunchKernelGGL(k_prescale2d, dim3((unsigned)cdiv((int64_t)d.V * d.Nu, 256)), dim3(256),
                       0, s, d, r, rs);
    INRCT_CHECK_LAUNCH();
    return rs;
}

void backproject(inrct_geom *geom, const float *r, float *v, hipStream_t s) {
    const GeomDev d = geom->dev();
    if (d.kind == INRCT_PAR2D || d.kind == INRCT_FAN2D) {
        const float *rs = prescale2d(geom, r, s);
        const dim3 grid((unsigned)cdiv(d.N, 8), (unsigned)cdiv(d.N, 8));
        if (d.kind == INRCT_FAN2D)
            hipLaunchKernelGGL(k_bproj2d<true>, grid, dim3(256), 0, s, d, rs, v);
        else
            hipLaunchKernelGGL(k_bproj2d<false>, grid, dim3(256), 0, s, d, rs, v);
        INRCT_CHECK_LAUNCH();
    } else {
        cone_backproject(geom, r, v, s);
    }
}

void backproject_at(inrct_geom *geom, const float *r, const int32_t *idx, int64_t k,
                    float *out, hipStream_t s) {
    if (k <= 0) return;
    if (geom->g.kind == INRCT_CONE3D) {
        cone_backproject_at(geom, r, idx, k, out, s);
        return;
    }
    const GeomDev d = geom->dev();
    const float *rs = prescale2d(geom, r, s);
    if (d.kind == INRCT_FAN2D)
        hipLaunchKernelGGL(k_bproj_at<true>, dim3((unsigned)cdiv(k, 256)), dim3(256), 0, s, d,
                           rs, idx, k, out);
    else
        hipLaunchKernelGGL(k_bproj_at<false>, dim3((unsigned)cdiv(k, 256)), dim3(256), 0, s, d,
                           rs, idx, k, out);
    INRCT_CHECK_LAUNCH();
}

void residual_loss(inrct_geom *geom, int loss, const float *z, const float *y,
                   float *r, double *loss_out, hipStream_t s) {
    const int64_t m = geom->m();
    const int nb = geom->n_partials;
    double *part = geom->partials.as<double>();
    if (loss == INRCT_LS) {
        hipLaunchKernelGGL(k_residual_ls, dim3(nb), dim3(256), 0, s, z, y, r, m, part);
        INRCT_CHECK_LAUNCH();
    } else {
        float *q = geom->q.as<float>();
        hipLaunchKernelGGL(k_diff, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, s, z, y,
                           q, m);
        INRCT_CHECK_LAUNCH();
        const int nu = geom->g.n_u;
        // the register-tiled filter: B outputs a thread (7, or more for wide
        // detectors), whole waves a row, as many rows a workgroup as fit
        int B = 7;
        while (B <= 13 && cdiv(nu, B) > 256) B += 2;
        if (B <= 13) {
            const int tpr = (int)(cdiv(cdiv(nu, B), 64) * 64);
            const int rpb = 256 / tpr;
            const size_t lds = sizeof(float) * ((size_t)(nu / 2) +
                                                (size_t)rpb * (3 * nu + 2 * kRampPad));
            const int64_t rows = m / nu;
#define RAMP_TILED(B_)                                                                    \
    hipLaunchKernelGGL(k_ramp_tiled<B_>, dim3(nb), dim3(256), lds, s, q, r, nu, rows, tpr, \
                       rpb, geom->g.du, part)
            if (B == 7) RAMP_TILED(7);
            else if (B == 9) RAMP_TILED(9);
            else if (B == 11) RAMP_TILED(11);
            else RAMP_TILED(13);
#undef RAMP_TILED
        } else {
            hipLaunchKernelGGL(k_ramp, dim3(nb), dim3(256), sizeof(float) * (3 * nu + nu / 2),
                               s, q, r, nu, m / nu, geom->g.du, part);
        }
        INRCT_CHECK_LAUNCH();
    }
    if (loss_out) launch_sum_partials(part, nb, loss_out, s);
}
}  // namespace inrct

namespace inrct {
// Argument checks of inrct_geom_create.
void check_geom_args(const ct_geometry *g, const inr_grid *grid) {
    INRCT_REQUIRE(g && grid, "null argument");
    INRCT_REQUIRE(grid->n >= 1 && grid->n <= 4096, "grid n must be in [1, 4096]");
    INRCT_REQUIRE(g->n_views >= 1 && g->n_u >= 1 && g->n_v >= 1, "empty detector");
    INRCT_REQUIRE(g->angles != nullptr, "angles must be a host array");
    INRCT_REQUIRE(g->du > 0 && g->dv > 0, "detector pitch must be positive");
    // the FLS filter stages a detector row (3.5 n_u floats) in 64 KB of LDS
    INRCT_REQUIRE(g->n_u <= 4096, "detector rows are limited to 4096 bins");
    if (g->kind == INRCT_PAR2D) {
        INRCT_REQUIRE(grid->dim == 2, "PAR2D needs a 2D grid");
        INRCT_REQUIRE(g->n_v == 1, "PAR2D needs n_v == 1");
    } else if (g->kind == INRCT_FAN2D) {
        INRCT_REQUIRE(grid->dim == 2, "FAN2D needs a 2D grid");
        INRCT_REQUIRE(g->n_v == 1, "FAN2D needs n_v == 1");
        // pixel segments reach sqrt(2) (1 + h) from the centre; the
        // adjoint's bin range needs the source beyond that
        INRCT_REQUIRE(g->sid > 1.4143 * (1.0 + 2.0 / grid->n) && g->idd > 0,
                      "source must lie outside the image");
    } else if (g->kind == INRCT_CONE3D) {
        INRCT_REQUIRE(grid->dim == 3, "CONE3D needs a 3D grid");
        INRCT_REQUIRE(g->sid > 1.8 && g->idd > 0, "source must lie outside the volume");
        // (every ray's z slope is checked per column when the tables are built)
        const double half_u = 0.5 * (g->n_u - 1) * g->du;
        INRCT_REQUIRE(half_u < 0.9 * (g->sid + g->idd),
                      "detector too wide for an in-plane principal axis");
    } else {
        set_error("unknown geometry kind %d", g->kind);
        throw Error{INRCT_ENOTSUP};
    }
}

inrct_geom *fresh_geom(const ct_geometry *g, const inr_grid *grid) {
    inrct_geom *h = new inrct_geom();
    h->g = *g;
    h->N = grid->n;
    h->dim = grid->dim;
    h->angles.assign(g->angles, g->angles + g->n_views);
    h->g.angles = h->angles.data();
    return h;
}

// Tables and scratch of a geometry handle, carved from `ar`.
void build_geom(inrct_geom *h, Arena &ar) {
    if (h->g.kind == INRCT_PAR2D || h->g.kind == INRCT_FAN2D) {
        std::vector<Col2D> cols;
        std::vector<float> steps;
        std::vector<View2D> views;
        build_tables(h->g, h->N, cols, steps, views);
        upload(ar, h->cols, cols);
        upload(ar, h->steps, steps);
        upload(ar, h->views, views);
        h->ut.alloc(ar, sizeof(float) * (size_t)h->N * h->N);
    } else {
        cone_build(h, ar);
    }
    const int64_t m = h->m();
    h->n_partials = (int)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(m, 4096)));
    h->partials.alloc(ar, sizeof(double) * h->n_partials);
    h->q.alloc(ar, sizeof(float) * m);
}
}  // namespace inrct

extern "C" {

int inrct_geom_create(const ct_geometry *g, const inr_grid *grid, void *ws, size_t ws_bytes,
                      hipStream_t stream, inrct_geom **out) {
    return guarded([&] {
        INRCT_REQUIRE(out, "null argument");
        *out = nullptr;
        check_geom_args(g, grid);
        inrct_geom *h = fresh_geom(g, grid);
        try {
            build_in_workspace(h, h->ws, ws, ws_bytes, stream,
                               [&] { return fresh_geom(g, grid); },
                               [](inrct_geom *x, Arena &ar) { build_geom(x, ar); });
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

int inrct_geom_destroy(inrct_geom *geom) {
    delete geom;
    return INRCT_OK;
}

int64_t inrct_geom_n_rays(const inrct_geom *geom) { return geom ? geom->m() : -1; }

int inrct_geom_adjoint_kind(const inrct_geom *geom) {
    if (!geom) return -1;
    if (geom->g.kind != INRCT_CONE3D) return INRCT_ADJ_2D;
    if (!geom->bp_lds) return INRCT_ADJ_DIRECT;
    return geom->bp_w2 ? INRCT_ADJ_WALK2 : INRCT_ADJ_WALK;
}

int ct_project(inrct_geom *geom, const float *u, float *z, hipStream_t stream) {
    return guarded([&] {
        INRCT_REQUIRE(geom && u && z, "null argument");
        project(geom, u, z, stream);
    });
}

int ct_backproject(inrct_geom *geom, const float *r, float *v, hipStream_t stream) {
    return guarded([&] {
        INRCT_REQUIRE(geom && r && v, "null argument");
        backproject(geom, r, v, stream);
    });
}

int ct_backproject_at(inrct_geom *geom, const float *r, const int32_t *idx, int64_t k,
                      float *v_out, hipStream_t stream) {
    return guarded([&] {
        INRCT_REQUIRE(geom && r && (k == 0 || (idx && v_out)), "null argument");
        INRCT_REQUIRE(k >= 0, "k must be >= 0");
        backproject_at(geom, r, idx, k, v_out, stream);
    });
}

int inrct_residual_loss(inrct_geom *geom, int loss, const float *z, const float *y,
                        float *r, double *loss_out, hipStream_t stream) {
    return guarded([&] {
        INRCT_REQUIRE(geom && z && y && r, "null argument");
        INRCT_REQUIRE(loss == INRCT_LS || loss == INRCT_FLS, "unknown loss %d", loss);
        residual_loss(geom, loss, z, y, r, loss_out, stream);
    });
}

}  // extern "C"
