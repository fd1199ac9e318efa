// Circular cone-beam Joseph projector P and its exact voxel-driven
// transpose (Sec. III: P in R^{m x n}; v = P^T r).
//
// For a flat detector whose row axis is the rotation axis, every ray of
// detector column a has the same in-plane direction, and the z position of
// ray (a, b) where it crosses slice s is affine in both s and b.  The host
// reduces each (view, column) to six 24.40 fixed-point integers in float64
// (see ConeCol); P and P^T evaluate the same integers, so P^T applies
// exactly the interpolation weights P applies, and neither does float64
// work per sample.
//
// P: one ray per lane, a wave an 8 x 8 patch of (column, row) rays and a
// workgroup 16 x 16, slices visited in
// order.  Rays whose principal axis is x read a transposed copy of the
// volume ([z][x][y]) so that neighbouring lanes read neighbouring addresses
// in both cases.
// P^T: one thread per (x, y) voxel column segment of kZc voxels; for each
// view, the detector columns whose stencil covers the voxel in-plane are
// found once per segment, then a monotone sweep over detector rows gathers
// the step-weighted residual for the kZc voxels.  No atomics.
#include <math.h>

#include "geom.h"

namespace inrct {

static const double kFix40 = 1099511627776.0;  // 2^40
static const int kPad = 2;  // zero border of the padded volume copies
static const unsigned kConeFwdLdsCap = 54 * 1024;  // occupancy cap of k_cone_fwd

// ------------------------------------------------------------------ host
void cone_build(inrct_geom *hd, Arena &ar) {
    const ct_geometry &g = hd->g;
    const int N = hd->N;
    const double h = 2.0 / N;
    const double c0 = -1.0 + 0.5 * h;
    const double tau = 1e-9;
    const double cv = 0.5 * (double)(g.n_v - 1);
    std::vector<ConeCol> cols((size_t)g.n_views * g.n_u);
    std::vector<ConeView> views(g.n_views);
    bool any_x = false;
    for (int j = 0; j < g.n_views; ++j) {
        const double cs = cos(g.angles[j]), sn = sin(g.angles[j]);
        ConeView &vg = views[j];
        vg.Sx = g.sid * cs;
        vg.Sy = g.sid * sn;
        vg.Cx = -g.idd * cs;
        vg.Cy = -g.idd * sn;
        vg.eux = -sn;
        vg.euy = cs;
        vg.any_x = vg.any_y = 0;
        const double Sz = 0.0, dz0 = 0.0;
        for (int a = 0; a < g.n_u; ++a) {
            const double ua = ((double)a - 0.5 * (double)(g.n_u - 1)) * g.du;
            const double dx = vg.Cx - vg.Sx + ua * vg.eux;
            const double dy = vg.Cy - vg.Sy + ua * vg.euy;
            ConeCol &c = cols[(size_t)j * g.n_u + a];
            c.ypr = fabs(dy) >= (1.0 - tau) * fabs(dx) ? 1 : 0;
            const double dax = c.ypr ? dy : dx, dot = c.ypr ? dx : dy;
            const double pax = c.ypr ? vg.Sy : vg.Sx, pot = c.ypr ? vg.Sx : vg.Sy;
            const double inv = 1.0 / dax;
            const double t0 = (c0 - pax) * inv;
            const double tN = t0 + (N - 1) * h * inv;
            INRCT_REQUIRE(t0 > 0 && tN > 0, "a grid slice lies behind the source");
            // Joseph needs every ray shallower in z than along its principal
            // axis; the steepest rays of the column are its end rows
            INRCT_REQUIRE(fabs(dz0) + cv * g.dv < fabs(dax),
                          "view %d column %d: the end rows are steeper in z than along the "
                          "principal axis (detector too tall)", j, a);
            const double phio = (pot + t0 * dot + 1.0) / h - 0.5;
            c.F0o = llrint(phio * kFix40);
            c.dFo = llrint(dot * inv * kFix40);
            const double Z0 = (Sz + t0 * dz0 + 1.0) / h - 0.5 - t0 * cv * g.dv / h;
            c.Z0 = llrint(Z0 * kFix40);
            c.D0 = llrint((inv * dz0 - inv * cv * g.dv) * kFix40);
            c.Z1 = llrint(t0 * g.dv / h * kFix40);
            c.D1 = llrint(inv * g.dv * kFix40);
            c.dxy2 = (float)(dx * dx + dy * dy);
            c.dz0 = (float)dz0;
            c.hinv = (float)(h * fabs(inv));
            if (c.ypr) vg.any_y = 1; else { vg.any_x = 1; any_x = true; }
        }
    }
    upload(ar, hd->ccols, cols);
    upload(ar, hd->cviews, views);
    hd->any_x = any_x;
    // zero-bordered copies of u in both layouts ([z][y][x] and [z][x][y]);
    // the border is cleared once here and never written afterwards
    const size_t Np = (size_t)N + 2 * kPad;
    // the projector addresses the padded copy with 32-bit element offsets
    INRCT_REQUIRE(Np * Np * Np < ((size_t)1 << 31), "cone-beam grid n = %d exceeds 1286", N);
    hd->ut.alloc(ar, sizeof(float) * Np * Np * Np * (any_x ? 2 : 1));
    zero_fill(ar, hd->ut);
}

// ---------------------------------------------------------------- device
// Workgroup id -> logical block: the hardware hands workgroups to the eight
// XCDs round-robin; each XCD is given a contiguous range of logical blocks
// so that blocks sharing volume or detector data run on the same L2.
__device__ __forceinline__ int xcd_block(int bid, int nb) {
    const int xcd = bid & 7, pos = bid >> 3;
    const int per = nb >> 3, rem = nb & 7;
    const int cnt = per + (xcd < rem ? 1 : 0);
    if (pos >= cnt) return -1;
    return xcd * per + (xcd < rem ? xcd : rem) + pos;
}

__device__ __forceinline__ int fx40_int(long long F) { return (int)(F >> 40); }
__device__ __forceinline__ float fx40_frac(long long F) {
    return (float)(unsigned int)(F >> 8) * 2.3283064365386963e-10f;
}

// Step length h |d| / |d_axis| of ray (column record c, row b), float32,
// written with explicitly rounded operations so P and P^T agree bitwise.
__device__ __forceinline__ float cone_step(const ConeDev &g, const ConeCol &c, int b) {
    const float vb = __fmul_rn(__fsub_rn((float)b, g.cvf), g.dvf);
    const float dz = __fadd_rn(c.dz0, vb);
    return __fmul_rn(c.hinv, __fsqrt_rn(__fadd_rn(c.dxy2, __fmul_rn(dz, dz))));
}

// Slices where floor(phi) in [-1, N - 1] (a superset; taps are bounds-checked).
__device__ __forceinline__ void range40(long long F0, long long dF, int N, int *lo, int *hi) {
    const double phi0 = (double)F0 * (1.0 / kFix40);
    const double sl = (double)dF * (1.0 / kFix40);
    double a, b;
    if (sl > 0) {
        a = (-1.0 - phi0) / sl;
        b = ((double)N - phi0) / sl;
    } else if (sl < 0) {
        a = ((double)N - phi0) / sl;
        b = (-1.0 - phi0) / sl;
    } else if (phi0 >= -1.0 && phi0 < (double)N) {
        a = 0;
        b = N - 1;
    } else {
        a = 1;
        b = 0;
    }
    double l = floor(a) - 1.0, r = ceil(b) + 1.0;
    if (l < 0) l = 0;
    if (r > N - 1) r = N - 1;
    *lo = (int)l;
    *hi = (int)r;
}

// The slice range [lo, hi] of range40 shrunk, with the exact fixed-point
// positions, to slices whose stencil index floor(phi) lies in [-1, N - 1]
// (phi is linear in s, so the valid slices form one interval).  Every tap
// of every visited slice then lies in [-1, N].
__device__ __forceinline__ void range40_exact(long long F0, long long dF, int N, int *lo,
                                              int *hi) {
    int l, r;
    range40(F0, dF, N, &l, &r);
    auto bad = [&](int s) {
        const int i = fx40_int(F0 + (long long)s * dF);
        return i < -1 || i > N - 1;
    };
    while (l <= r && bad(l)) ++l;
    while (r >= l && bad(r)) --r;
    *lo = l;
    *hi = r;
}

// up[z+kPad][y+kPad][x+kPad] = u[z][y][x] and (if ut) ut[z+kPad][x+kPad][y+kPad] = u[z][y][x]
__global__ __launch_bounds__(256) void k_pad_copy(const float *__restrict__ u,
                                                  float *__restrict__ up,
                                                  float *__restrict__ ut, int N) {
    __shared__ float tile[32][33];
    const int Np = N + 2 * kPad;
    const int z = blockIdx.z;
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    const size_t base = (size_t)z * N * N;
    const size_t pbase = (size_t)(z + kPad) * Np * Np;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int y = y0 + k, x = x0 + tx;
        if (x < N && y < N) {
            const float val = u[base + (size_t)y * N + x];
            tile[k][tx] = val;
            up[pbase + (size_t)(y + kPad) * Np + x + kPad] = val;
        }
    }
    if (ut == nullptr) return;
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int x = x0 + k, y = y0 + tx;
        if (x < N && y < N) ut[pbase + (size_t)(x + kPad) * Np + y + kPad] = tile[tx][k];
    }
}

// One ray per lane.  Reads the zero-bordered copies: over the exact slice
// range every tap index lies in [-1, N], inside the kPad-wide zero border,
// so no tap needs a bounds test.
__global__ __launch_bounds__(256) void k_cone_fwd(ConeDev g, const float *__restrict__ up,
                                                  const float *__restrict__ utp,
                                                  float *__restrict__ z, int ncx, int ncy) {
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    if (lb < 0) return;
    // a wave is an 8 x 8 patch of rays (columns x rows); a block 16 x 16.
    // Blocks go in pairs of row tiles, column tiles next, then row-tile
    // pairs, then views: both tiles that share a boundary row of voxels,
    // and the tiles beside them, run at about the same time.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ngr = (ncy + 1) >> 1;
    const int rt = ((lb / (2 * ncx)) % ngr) * 2 + (lb & 1);
    const int a = ((lb >> 1) % ncx) * 16 + (wave & 1) * 8 + (lane & 7);
    const int b = rt * 16 + (wave >> 1) * 8 + (lane >> 3);
    const int j = lb / (2 * ncx * ngr);
    if (a >= g.Nu || b >= g.Nv) return;
    const ConeCol c = g.col[(size_t)j * g.Nu + a];
    const long long F0z = c.Z0 + (long long)b * c.Z1;
    const long long dFz = c.D0 + (long long)b * c.D1;
    const int N = g.N;
    const int Np = N + 2 * kPad, Np2 = Np * Np;
    int lo1, hi1, lo2, hi2;
    range40_exact(c.F0o, c.dFo, N, &lo1, &hi1);
    range40_exact(F0z, dFz, N, &lo2, &hi2);
    const int lo = max(lo1, lo2), hi = min(hi1, hi2);
    const float *__restrict__ src = c.ypr ? up : utp;
    long long Fo = c.F0o + (long long)lo * c.dFo;
    long long Fz = F0z + (long long)lo * dFz;
    // element offset of tap (iz, s, io): (iz + kPad) Np2 + (s + kPad) Np + io + kPad
    int srow = (lo + kPad) * Np + kPad * Np2 + kPad;
    float acc = 0.f;
    // Four steps per iteration, all taps loaded before any is used, so each
    // wave keeps sixteen gathers in flight; the sum stays in step order.
    int s = lo;
    for (; s + 3 <= hi; s += 4) {
        float v[4][4], wo[4], wz[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const long long Foq = Fo + q * c.dFo, Fzq = Fz + q * dFz;
            const int e = srow + q * Np + fx40_int(Fzq) * Np2 + fx40_int(Foq);
            wo[q] = fx40_frac(Foq);
            wz[q] = fx40_frac(Fzq);
            v[q][0] = src[e];
            v[q][1] = src[e + 1];
            v[q][2] = src[e + Np2];
            v[q][3] = src[e + Np2 + 1];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc += (1.f - wz[q]) * ((1.f - wo[q]) * v[q][0] + wo[q] * v[q][1]) +
                   wz[q] * ((1.f - wo[q]) * v[q][2] + wo[q] * v[q][3]);
        Fo += 4 * c.dFo;
        Fz += 4 * dFz;
        srow += 4 * Np;
    }
    for (; s <= hi; ++s, Fo += c.dFo, Fz += dFz, srow += Np) {
        const int io = fx40_int(Fo), iz = fx40_int(Fz);
        const float wo = fx40_frac(Fo), wz = fx40_frac(Fz);
        const int e = srow + iz * Np2 + io;
        const float v00 = src[e], v01 = src[e + 1];
        const float v10 = src[e + Np2], v11 = src[e + Np2 + 1];
        acc += (1.f - wz) * ((1.f - wo) * v00 + wo * v01) + wz * ((1.f - wo) * v10 + wo * v11);
    }
    z[((size_t)j * g.Nv + b) * g.Nu + a] = acc * cone_step(g, c, b);
}

// rs = r * step length (applied on the ray side of P^T)
__global__ __launch_bounds__(256) void k_cone_prescale(ConeDev g, const float *__restrict__ r,
                                                       float *__restrict__ rs) {
    const int a = blockIdx.x * 64 + (threadIdx.x & 63);
    const int b = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int j = blockIdx.z;
    if (a >= g.Nu || b >= g.Nv) return;
    const size_t i = ((size_t)j * g.Nv + b) * g.Nu + a;
    rs[i] = r[i] * cone_step(g, g.col[(size_t)j * g.Nu + a], b);
}

// Columns whose ray crosses the in-plane segment p1-p2: those at positions
// between the central projections of its end points.  Computed in single precision and
// widened by a margin far above its rounding error: the caller tests every
// candidate exactly, so extra columns cost time but never change a sum.
__device__ __forceinline__ void cone_cols(const ConeDev &g, const ConeView &vg, float p1x,
                                          float p1y, float p2x, float p2y, int *lo, int *hi) {
    const float ax = (float)(vg.Sx - vg.Cx), ay = (float)(vg.Sy - vg.Cy);
    const float sx = (float)vg.Sx, sy = (float)vg.Sy;
    const float eux = (float)vg.eux, euy = (float)vg.euy;
    const float D1x = p1x - sx, D1y = p1y - sy;
    const float D2x = p2x - sx, D2y = p2y - sy;
    // hardware reciprocal (about 1 ulp): far inside the 0.01-column margin
    const float u1 = (ax * D1y - ay * D1x) * __builtin_amdgcn_rcpf(eux * D1y - euy * D1x);
    const float u2 = (ax * D2y - ay * D2x) * __builtin_amdgcn_rcpf(eux * D2y - euy * D2x);
    const float c = 0.5f * (float)(g.Nu - 1);
    const float a1 = u1 / (float)g.du + c, a2 = u2 / (float)g.du + c;
    // the columns inside [a1, a2], widened by the margin
    float l = ceilf(fminf(a1, a2) - 0.01f), r = floorf(fmaxf(a1, a2) + 0.01f);
    l = fmaxf(l, 0.f);
    r = fminf(r, (float)(g.Nu - 1));
    *lo = (int)l;
    *hi = (int)r;
}

// (P^T r) for voxels (ix, iy, z0 .. z0 + ZC - 1), accumulated into acc.
// rs is the step-weighted residual.
template <int ZC>
__device__ __forceinline__ void cone_gather(const ConeDev &g, const float *__restrict__ rs,
                                            int ix, int iy, int z0, float (&acc)[ZC]) {
    const float h = (float)g.h;
    const float x = (float)(-1.0 + (ix + 0.5) * g.h), y = (float)(-1.0 + (iy + 0.5) * g.h);
    const int Nu = g.Nu, Nv = g.Nv;
    for (int j = 0; j < g.V; ++j) {
        const ConeView vg = g.view[j];
        const float *rj = rs + (size_t)j * Nv * Nu;
        for (int pass = 0; pass < 2; ++pass) {
            const bool ypass = pass == 0;
            if (ypass ? !vg.any_y : !vg.any_x) continue;
            const int s = ypass ? iy : ix, o = ypass ? ix : iy;
            int lo, hi;
            if (ypass) cone_cols(g, vg, x - h, y, x + h, y, &lo, &hi);
            else cone_cols(g, vg, x, y - h, x, y + h, &lo, &hi);
            for (int a = lo; a <= hi; ++a) {
                const ConeCol c = g.col[(size_t)j * Nu + a];
                if ((c.ypr != 0) != ypass) continue;
                const long long Fo = c.F0o + (long long)s * c.dFo;
                const int io = fx40_int(Fo);
                if (io != o && io != o - 1) continue;
                const float fo = fx40_frac(Fo);
                const float wo = io == o ? 1.f - fo : fo;
                const long long E0 = c.Z0 + (long long)s * c.D0;
                const long long E1 = c.Z1 + (long long)s * c.D1;  // > 0
                // first row whose stencil reaches z0 - 1
                const long long lo_t = (long long)(z0 - 1) << 40;
                // row estimate in single precision; the walks below make it exact
                float bd = floorf((float)(lo_t - E0) * __builtin_amdgcn_rcpf((float)E1)) - 1.f;
                bd = bd < 0.f ? 0.f : (bd > (float)Nv ? (float)Nv : bd);
                int b = (int)bd;
                long long ph = E0 + (long long)b * E1;
                while (b > 0 && ph - E1 >= lo_t) {
                    --b;
                    ph -= E1;
                }
                while (b < Nv && ph < lo_t) {
                    ++b;
                    ph += E1;
                }
                // One pass over the rows from b on: a row whose stencil
                // starts at voxel i0 gives (1 - w) to i0 and w to i0 + 1.
                // Every voxel still receives its terms in increasing row
                // order with the same products, so the sums are unchanged.
                const float *rp = rj + a + (size_t)b * Nu;
                while (b < Nv && fx40_int(ph) == z0 - 1) {
                    acc[0] += wo * fx40_frac(ph) * rp[0];
                    ++b;
                    ph += E1;
                    rp += Nu;
                }
#pragma unroll
                for (int jz = 0; jz < ZC; ++jz) {
                    while (b < Nv && fx40_int(ph) == z0 + jz) {
                        const float w = fx40_frac(ph);
                        const float r = rp[0];
                        acc[jz] += wo * (1.f - w) * r;
                        if (jz + 1 < ZC) acc[jz + 1] += wo * w * r;
                        ++b;
                        ph += E1;
                        rp += Nu;
                    }
                }
            }
        }
    }
}

constexpr int kZc = 16;

__global__ __launch_bounds__(256) void k_cone_bp(ConeDev g, const float *__restrict__ rs,
                                                 float *__restrict__ v, int nbx, int nby) {
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    if (lb < 0) return;
    // a wave is an 8 x 8 patch of (x, y) voxel columns; a block 16 x 16
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ix = (lb % nbx) * 16 + (wave & 1) * 8 + (lane & 7);
    const int iy = ((lb / nbx) % nby) * 16 + (wave >> 1) * 8 + (lane >> 3);
    const int z0 = (lb / (nbx * nby)) * kZc;
    if (ix >= g.N || iy >= g.N) return;
    float acc[kZc];
#pragma unroll
    for (int i = 0; i < kZc; ++i) acc[i] = 0.f;
    cone_gather<kZc>(g, rs, ix, iy, z0, acc);
    const size_t NN = (size_t)g.N * g.N;
#pragma unroll
    for (int i = 0; i < kZc; ++i)
        if (z0 + i < g.N) v[(size_t)(z0 + i) * NN + (size_t)iy * g.N + ix] = acc[i];
}

__global__ __launch_bounds__(256) void k_cone_bp_at(ConeDev g, const float *__restrict__ rs,
                                                    const int32_t *__restrict__ idx, int64_t k,
                                                    float *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= k) return;
    const int64_t q = idx[t];
    const int N = g.N;
    float acc[1] = {0.f};
    cone_gather<1>(g, rs, (int)(q % N), (int)((q / N) % N), (int)(q / ((int64_t)N * N)), acc);
    out[t] = acc[0];
}

// ----------------------------------------------------------- host wrappers
void cone_project(inrct_geom *hd, const float *u, float *z, hipStream_t s) {
    const ConeDev d = hd->cone();
    const size_t Np = (size_t)d.N + 2 * kPad;
    float *up = hd->ut.as<float>();
    float *utp = hd->any_x ? up + Np * Np * Np : up;
    hipLaunchKernelGGL(k_pad_copy, dim3((unsigned)cdiv(d.N, 32), (unsigned)cdiv(d.N, 32), d.N),
                       dim3(256), 0, s, u, up, hd->any_x ? utp : nullptr, d.N);
    INRCT_CHECK_LAUNCH();
    const int ncx = (int)cdiv(d.Nu, 16), ncy = (int)cdiv(d.Nv, 16);
    const int ngr = (ncy + 1) / 2;  // row-tile pairs (the last may be half empty)
    // The launch reserves 54 KB of LDS it does not use, so that at most two
    // blocks share a CU: with fewer rays in flight per XCD, the voxel lines a
    // block fetches are still in L2 when the neighbouring blocks read them
    // (10.3 -> 8.6 ms at 501^3; four blocks per CU 9.7 ms, three 9.3 ms, one
    // 12.5 ms).
    hipLaunchKernelGGL(k_cone_fwd, dim3((unsigned)(ncx * ngr * 2 * d.V)), dim3(256),
                       kConeFwdLdsCap, s, d, up, utp, z, ncx, ncy);
    INRCT_CHECK_LAUNCH();
}

static const float *cone_prescale(inrct_geom *hd, const float *r, hipStream_t s) {
    const ConeDev d = hd->cone();
    float *rs = hd->q.as<float>();
    hipLaunchKernelGGL(k_cone_prescale, dim3((unsigned)cdiv(d.Nu, 64), (unsigned)cdiv(d.Nv, 4), d.V),
                       dim3(256), 0, s, d, r, rs);
    INRCT_CHECK_LAUNCH();
    return rs;
}

void cone_backproject(inrct_geom *hd, const float *r, float *v, hipStream_t s) {
    const float *rs = cone_prescale(hd, r, s);
    const ConeDev d = hd->cone();
    const int nbx = (int)cdiv(d.N, 16), nby = (int)cdiv(d.N, 16), nbz = (int)cdiv(d.N, kZc);
    hipLaunchKernelGGL(k_cone_bp, dim3((unsigned)(nbx * nby * nbz)), dim3(256), 0, s, d, rs, v,
                       nbx, nby);
    INRCT_CHECK_LAUNCH();
}

void cone_backproject_at(inrct_geom *hd, const float *r, const int32_t *idx, int64_t k,
                         float *out, hipStream_t s) {
    const float *rs = cone_prescale(hd, r, s);
    const ConeDev d = hd->cone();
    hipLaunchKernelGGL(k_cone_bp_at, dim3((unsigned)cdiv(k, 256)), dim3(256), 0, s, d, rs, idx, k,
                       out);
    INRCT_CHECK_LAUNCH();
}

}  // namespace inrct
