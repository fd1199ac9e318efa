// 2D parallel-beam Joseph projector P, its voxel-driven exact transpose P^T,
// the data-fidelity residuals (Sec. II, Sec. III of the paper) and the
// geometry handle.  The cone-beam kernels are in cone.hip.
//
// Geometry is reduced on the host, in float64, to one record per (view,
// detector bin): the principal axis, 1/d_axis, the ray parameter at the
// first slice and the interpolation position of the in-plane "other"
// coordinate as a 32.32 fixed-point start value and per-slice increment.
// Because the interpolation position at slice s is the exact integer
// F0 + s * dF in both kernels, P^T applies exactly the weights P applies.
#include <math.h>

#include "geom.h"

namespace inrct {

static const double kFix = 4294967296.0;       // 2^32
static const float kInvFix = 2.3283064365386963e-10f;  // 2^-32

// ------------------------------------------------------------- host tables
static void build_tables(const ct_geometry &g, int N, std::vector<ColGeom> &cols,
                         std::vector<ViewGeom> &views) {
    const double h = 2.0 / N;
    const double c0 = -1.0 + 0.5 * h;
    const double tau = 1e-9;
    cols.resize((size_t)g.n_views * g.n_u);
    views.resize(g.n_views);
    for (int j = 0; j < g.n_views; ++j) {
        const double th = g.angles[j];
        const double cs = cos(th), sn = sin(th);
        ViewGeom &vg = views[j];
        vg.cs = cs;
        vg.sn = sn;
        vg.any_x = vg.any_y = 0;
        if (g.kind != INRCT_PAR2D) {  // fan (and the in-plane part of cone)
            vg.Sx = g.sid * cs;
            vg.Sy = g.sid * sn;
            vg.Cx = -g.idd * cs;
            vg.Cy = -g.idd * sn;
            vg.eux = -sn;
            vg.euy = cs;
        } else {
            vg.Sx = vg.Sy = vg.Cx = vg.Cy = 0.0;
            vg.eux = cs;
            vg.euy = sn;
        }
        for (int a = 0; a < g.n_u; ++a) {
            const double ua = ((double)a - 0.5 * (double)(g.n_u - 1)) * g.du;
            double p0x, p0y, p0z, dx, dy, dz0;
            if (g.kind != INRCT_PAR2D) {
                p0x = vg.Sx;
                p0y = vg.Sy;
                p0z = 0.0;
                dx = vg.Cx - vg.Sx + ua * vg.eux;
                dy = vg.Cy - vg.Sy + ua * vg.euy;
                dz0 = 0.0;
            } else {
                p0x = ua * cs;
                p0y = ua * sn;
                p0z = 0.0;
                dx = -sn;
                dy = cs;
                dz0 = 0.0;
            }
            ColGeom &c = cols[(size_t)j * g.n_u + a];
            c.ypr = fabs(dy) >= (1.0 - tau) * fabs(dx) ? 1 : 0;
            const double dax = c.ypr ? dy : dx;
            const double dot = c.ypr ? dx : dy;
            const double pax = c.ypr ? p0y : p0x;
            const double pot = c.ypr ? p0x : p0y;
            c.inv = 1.0 / dax;
            c.t0 = (c0 - pax) * c.inv;
            const double phi0 = (pot + c.t0 * dot + 1.0) / h - 0.5;
            c.F0o = llrint(phi0 * kFix);
            c.dFo = llrint(dot * c.inv * kFix);
            c.p0z = p0z;
            c.dz0 = dz0;
            c.dxy2 = dx * dx + dy * dy;
            c.pad = 0;
            if (c.ypr) vg.any_y = 1; else vg.any_x = 1;
        }
    }
}

// --------------------------------------------------------- device helpers
__device__ __forceinline__ float ray_step2d(const GeomDev &g, const ColGeom &c) {
#pragma clang fp contract(off)
    return (float)(g.h * sqrt(c.dxy2) * fabs(c.inv));
}

__device__ __forceinline__ int fx_int(long long F) { return (int)(F >> 32); }
__device__ __forceinline__ float fx_frac(long long F) {
    return (float)(unsigned int)(F & 0xffffffffLL) * kInvFix;
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
__global__ __launch_bounds__(256) void k_proj2d(GeomDev g, const float *__restrict__ u,
                                                float *__restrict__ z) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (k >= g.Nu) return;
    const ColGeom c = g.col[(size_t)j * g.Nu + k];
    const int N = g.N;
    int lo, hi;
    slice_range(c.F0o, c.dFo, N, &lo, &hi);
    long long F = c.F0o + (long long)lo * c.dFo;
    float acc = 0.f;
    for (int s = lo; s <= hi; ++s, F += c.dFo) {
        const int io = fx_int(F);
        const float w = fx_frac(F);
        float v0 = 0.f, v1 = 0.f;
        const size_t base = c.ypr ? (size_t)s * N : (size_t)s;
        const size_t str = c.ypr ? 1 : (size_t)N;
        if ((unsigned)io < (unsigned)N) v0 = u[base + (size_t)io * str];
        if ((unsigned)(io + 1) < (unsigned)N) v1 = u[base + (size_t)(io + 1) * str];
        acc += (1.f - w) * v0 + w * v1;
    }
    z[(size_t)j * g.Nu + k] = acc * ray_step2d(g, c);
}

// ------------------------------------------------ adjoint (gather) helpers
__device__ __forceinline__ void par_col_range(const GeomDev &g, const ViewGeom &vg,
                                              double p1x, double p1y, double p2x,
                                              double p2y, int *lo, int *hi) {
    const double s1 = p1x * vg.cs + p1y * vg.sn, s2 = p2x * vg.cs + p2y * vg.sn;
    const double c = 0.5 * (double)(g.Nu - 1);
    const double a1 = s1 / g.du + c, a2 = s2 / g.du + c;
    double l = floor(fmin(a1, a2)), r = ceil(fmax(a1, a2));
    if (l < 0) l = 0;
    if (r > g.Nu - 1) r = g.Nu - 1;
    *lo = (int)l;
    *hi = (int)r;
}

// Fan beam: bins whose ray crosses the in-plane segment p1-p2 (central
// projection of the end points from the source onto the detector line,
// widened by 1e-6 bin against rounding, then rounded outwards).  The
// projection is monotone along the segment because the whole segment lies
// on the detector's side of the line through the source parallel to it.
__device__ __forceinline__ void fan_col_range(const GeomDev &g, const ViewGeom &vg,
                                              double p1x, double p1y, double p2x,
                                              double p2y, int *lo, int *hi) {
    const double ax = vg.Sx - vg.Cx, ay = vg.Sy - vg.Cy;
    const double D1x = p1x - vg.Sx, D1y = p1y - vg.Sy;
    const double D2x = p2x - vg.Sx, D2y = p2y - vg.Sy;
    const double u1 = (ax * D1y - ay * D1x) / (vg.eux * D1y - vg.euy * D1x);
    const double u2 = (ax * D2y - ay * D2x) / (vg.eux * D2y - vg.euy * D2x);
    const double c = 0.5 * (double)(g.Nu - 1);
    const double a1 = u1 / g.du + c, a2 = u2 / g.du + c;
    double l = floor(fmin(a1, a2) - 1e-6), r = ceil(fmax(a1, a2) + 1e-6);
    if (l < 0) l = 0;
    if (r > g.Nu - 1) r = g.Nu - 1;
    *lo = (int)l;
    *hi = (int)r;
}

// weight of voxel index `o` in the linear stencil at position F
__device__ __forceinline__ float stencil_weight(long long F, int o, bool *hit) {
    const int i0 = fx_int(F);
    const float w = fx_frac(F);
    *hit = true;
    if (i0 == o) return 1.f - w;
    if (i0 == o - 1) return w;
    *hit = false;
    return 0.f;
}

// (P^T r) at pixel (ix, iy) of a 2D parallel- or fan-beam geometry.
__device__ float bp_pixel_2d(const GeomDev &g, const float *__restrict__ r, int ix,
                             int iy) {
    const double h = g.h;
    const double x = -1.0 + (ix + 0.5) * h, y = -1.0 + (iy + 0.5) * h;
    float acc = 0.f;
    for (int j = 0; j < g.V; ++j) {
        const ViewGeom vg = g.view[j];
        const float *rj = r + (size_t)j * g.Nu;
        for (int pass = 0; pass < 2; ++pass) {
            const bool ypass = pass == 0;
            if (ypass ? !vg.any_y : !vg.any_x) continue;
            const int s = ypass ? iy : ix, o = ypass ? ix : iy;
            int lo, hi;
            if (g.kind == INRCT_FAN2D) {
                if (ypass) fan_col_range(g, vg, x - h, y, x + h, y, &lo, &hi);
                else fan_col_range(g, vg, x, y - h, x, y + h, &lo, &hi);
            } else {
                if (ypass) par_col_range(g, vg, x - h, y, x + h, y, &lo, &hi);
                else par_col_range(g, vg, x, y - h, x, y + h, &lo, &hi);
            }
            for (int k = lo; k <= hi; ++k) {
                const ColGeom c = g.col[(size_t)j * g.Nu + k];
                if ((c.ypr != 0) != ypass) continue;
                bool hit;
                const float w = stencil_weight(c.F0o + (long long)s * c.dFo, o, &hit);
                if (hit) acc += w * ray_step2d(g, c) * rj[k];
            }
        }
    }
    return acc;
}

__global__ __launch_bounds__(256) void k_bproj2d(GeomDev g, const float *__restrict__ r,
                                                 float *__restrict__ v) {
    const int ix = blockIdx.x * 64 + (threadIdx.x & 63);
    const int iy = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (ix >= g.N || iy >= g.N) return;
    v[(size_t)iy * g.N + ix] = bp_pixel_2d(g, r, ix, iy);
}

__global__ __launch_bounds__(256) void k_bproj_at(GeomDev g, const float *__restrict__ r,
                                                  const int32_t *__restrict__ idx,
                                                  int64_t k, float *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= k) return;
    const int64_t q = idx[t];
    const int N = g.N;
    out[t] = bp_pixel_2d(g, r, (int)(q % N), (int)((q / N) % N));
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
// per-block partials of 1/2 q.r.  Row length nu, rows = m / nu.
__global__ __launch_bounds__(256) void k_ramp(const float *__restrict__ q, float *r,
                                              int nu, int64_t rows, double du,
                                              double *partials) {
    __shared__ double sh[256];
    double acc = 0.0;
    const int64_t m = rows * nu;
    const float f0 = (float)(1.0 / (4.0 * du));
    const float cf = (float)(-1.0 / (M_PI * M_PI * du));
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += stride) {
        const int64_t row = i / nu;
        const int a = (int)(i - row * nu);
        const float *qr = q + row * nu;
        float s = f0 * qr[a];
        // odd offsets only: f_j = -1/(pi^2 j^2 du)
        for (int jj = 1; jj < nu; jj += 2) {
            float t = 0.f;
            if (a - jj >= 0) t += qr[a - jj];
            if (a + jj < nu) t += qr[a + jj];
            s += cf / ((float)jj * (float)jj) * t;
        }
        r[i] = s;
        acc += 0.5 * (double)qr[a] * (double)s;
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

void project(inrct_geom *geom, const float *u, float *z, hipStream_t s) {
    const GeomDev d = geom->dev();
    if (d.kind == INRCT_PAR2D || d.kind == INRCT_FAN2D) {
        hipLaunchKernelGGL(k_proj2d, dim3((unsigned)cdiv(d.Nu, 256), d.V), dim3(256),
                           0, s, d, u, z);
        INRCT_CHECK_LAUNCH();
    } else {
        cone_project(geom, u, z, s);
    }
}

void backproject(inrct_geom *geom, const float *r, float *v, hipStream_t s) {
    const GeomDev d = geom->dev();
    if (d.kind == INRCT_PAR2D || d.kind == INRCT_FAN2D) {
        hipLaunchKernelGGL(k_bproj2d, dim3((unsigned)cdiv(d.N, 64), (unsigned)cdiv(d.N, 4)),
                           dim3(256), 0, s, d, r, v);
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
    hipLaunchKernelGGL(k_bproj_at, dim3((unsigned)cdiv(k, 256)), dim3(256), 0, s, d, r,
                       idx, k, out);
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
        hipLaunchKernelGGL(k_ramp, dim3(nb), dim3(256), 0, s, q, r, geom->g.n_u,
                           m / geom->g.n_u, geom->g.du, part);
        INRCT_CHECK_LAUNCH();
    }
    if (loss_out) launch_sum_partials(part, nb, loss_out, s);
}
}  // namespace inrct

extern "C" {

int inrct_geom_create(const ct_geometry *g, const inr_grid *grid, inrct_geom **out) {
    return guarded([&] {
        INRCT_REQUIRE(g && grid && out, "null argument");
        *out = nullptr;
        INRCT_REQUIRE(grid->n >= 1 && grid->n <= 4096, "grid n must be in [1, 4096]");
        INRCT_REQUIRE(g->n_views >= 1 && g->n_u >= 1 && g->n_v >= 1, "empty detector");
        INRCT_REQUIRE(g->angles != nullptr, "angles must be a host array");
        INRCT_REQUIRE(g->du > 0 && g->dv > 0, "detector pitch must be positive");
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
            // every ray must be shallower in z than in-plane
            const double half_v = 0.5 * (g->n_v - 1) * g->dv;
            const double half_u = 0.5 * (g->n_u - 1) * g->du;
            const double dmin = sqrt((g->sid + g->idd) * (g->sid + g->idd));
            INRCT_REQUIRE(half_v < 0.9 * dmin && half_u < 0.9 * dmin,
                          "detector too large for an in-plane principal axis");
        } else {
            set_error("unknown geometry kind %d", g->kind);
            throw Error{INRCT_ENOTSUP};
        }
        inrct_geom *h = new inrct_geom();
        try {
            h->g = *g;
            h->N = grid->n;
            h->dim = grid->dim;
            h->angles.assign(g->angles, g->angles + g->n_views);
            h->g.angles = h->angles.data();
            if (g->kind == INRCT_PAR2D || g->kind == INRCT_FAN2D) {
                std::vector<ColGeom> cols;
                std::vector<ViewGeom> views;
                build_tables(h->g, h->N, cols, views);
                upload(h->cols, cols);
                upload(h->views, views);
            } else {
                cone_build(h);
            }
            const int64_t m = h->m();
            h->n_partials = (int)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(m, 4096)));
            h->partials.alloc(sizeof(double) * h->n_partials);
            h->q.alloc(sizeof(float) * m);
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
