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
// P: a workgroup integrates a tile of 64 x 24 rays of one view, slice chunk
// by slice chunk, from the chunk's footprint of u staged in LDS.
// P^T: one thread per (x, y) voxel column segment of kZc voxels; view by
// view the block's detector footprint is staged in LDS; the detector
// columns whose stencil covers the voxel in-plane are found once per
// segment, then a monotone sweep over detector rows gathers the
// step-weighted residual for the kZc voxels.  No atomics.
#include <math.h>

#include "geom.h"

namespace inrct {

static const double kFix40 = 1099511627776.0;  // 2^40

// LDS footprint of one chunk of a projector tile: at most kFootO positions
// along the ray's non-principal in-plane axis and kFootZ along z.  Two
// layouts (floats):
//   y-principal rays, [s][z][o]: o stride 1, z stride kLdsZY, s stride
//     kFootZ kLdsZY (rows padded to 65 so neighbouring z rows fall in
//     neighbouring banks);
//   x-principal rays, [o][z][s]: s stride 1, z stride kLdsZX, o stride
//     kLdsOX (odd, so lanes at neighbouring o hit neighbouring banks);
// each matching the direction in which u ([z][y][x]) is contiguous.
constexpr int kFootO = 80, kFootZ = 24;
// The adjoint: voxels per thread along z, and the LDS footprint caps
// (detector columns and rows per view and block) with the staged row stride
constexpr int kZc = 16;
constexpr int kBpA = 64, kBpB = 48, kBpRs = kBpA + 1;
constexpr int kLdsZY = kFootO + 1, kLdsSY = kFootZ * kLdsZY;
constexpr int kLdsZX = kTileS, kLdsOX = kFootZ * kLdsZX + 1;
constexpr int kLdsFloatsY = kTileS * kLdsSY, kLdsFloatsX = kFootO * kLdsOX;

__host__ __device__ inline int fx40_floor(long long F) { return (int)(F >> 40); }

// Extents of a chunk's footprint.  The interpolation positions are
// monotone in the detector column, row and slice (each ray is a line, the
// rays of a tile are ordered), so their extremes over the tile and the
// chunk's kTileS slices are attained at the corners; one voxel of margin on
// each side absorbs the fixed-point rounding.  Every tap (i, i + 1) of every
// ray of the tile then lies in [lo, lo + extent).  Host and device run this
// same integer arithmetic.
struct Footprint {
    int olo, oext, zlo, zext;
};

// The tile's corner positions at the first and last slice of a chunk (4
// along the other axis, 8 along z), advanced from chunk to chunk by exact
// integer steps.
struct Corners {
    long long o[4], z[8];
    long long dO[4], dZ[8];  // per-slice steps
    __host__ __device__ void init(const ConeCol &ca, const ConeCol &cb, int b0, int b1, int s0) {
        const ConeCol *cc[2] = {&ca, &cb};
        for (int q = 0; q < 2; ++q)
            for (int e = 0; e < 2; ++e) {
                const long long s = s0 + (e ? kTileS - 1 : 0);
                const ConeCol &c = *cc[q];
                o[2 * q + e] = c.F0o + s * c.dFo;
                dO[2 * q + e] = c.dFo;
                for (int f = 0; f < 2; ++f) {
                    const long long b = f ? b1 : b0;
                    dZ[4 * q + 2 * e + f] = c.D0 + b * c.D1;
                    z[4 * q + 2 * e + f] = c.Z0 + b * c.Z1 + s * dZ[4 * q + 2 * e + f];
                }
            }
    }
    __host__ __device__ void advance() {
        for (int i = 0; i < 4; ++i) o[i] += kTileS * dO[i];
        for (int i = 0; i < 8; ++i) z[i] += kTileS * dZ[i];
    }
    __host__ __device__ Footprint footprint() const {
        int omin = fx40_floor(o[0]), omax = omin, zmin = fx40_floor(z[0]), zmax = zmin;
        for (int i = 1; i < 4; ++i) {
            const int v = fx40_floor(o[i]);
            omin = v < omin ? v : omin;
            omax = v > omax ? v : omax;
        }
        for (int i = 1; i < 8; ++i) {
            const int v = fx40_floor(z[i]);
            zmin = v < zmin ? v : zmin;
            zmax = v > zmax ? v : zmax;
        }
        Footprint f;
        f.olo = omin - 1;
        f.oext = omax - omin + 4;  // taps up to omax + 1, one position of margin each side
        f.zlo = zmin - 1;
        f.zext = zmax - zmin + 4;
        return f;
    }
};

// Slices s in [0, N) where the ray's interpolation index floor(phi(s)) lies
// in [-1, N - 1], phi(s) = F0 + s dF (a superset from float64, widened by
// one slice; the empty set is lo > hi).
static void valid_slices(long long F0, long long dF, int N, int *lo, int *hi) {
    const double phi0 = (double)F0 / kFix40, sl = (double)dF / kFix40;
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
        *lo = 1;
        *hi = 0;
        return;
    }
    const double l = std::max(0.0, floor(a) - 1.0), r = std::min((double)N - 1, ceil(b) + 1.0);
    *lo = (int)l;
    *hi = (int)r;
}

// Slices where the in-plane path of column record c passes within radius
// 1 + 2h of the rotation axis: outside them both taps of the slice lie
// outside the FOV cylinder (centres farther than 1 from the axis), where an
// image produced on the FOV vanishes.
static void fov_slices(const ConeCol &c, int N, int *lo, int *hi) {
    const double h = 2.0 / N, R = 1.0 + 2.0 * h;
    // slice coordinate -1 + (s + 1/2) h; other coordinate -1 + (phi + 1/2) h
    const double p0 = (double)c.F0o / kFix40, sl = (double)c.dFo / kFix40;
    const double ao = sl * h, bo = -1.0 + (p0 + 0.5) * h;  // other = ao s + bo
    const double as = h, bs = -1.0 + 0.5 * h;              // slice = as s + bs
    const double A = ao * ao + as * as, B = 2.0 * (ao * bo + as * bs),
                 C = bo * bo + bs * bs - R * R;
    const double disc = B * B - 4.0 * A * C;
    if (disc <= 0) {
        *lo = 1;
        *hi = 0;
        return;
    }
    const double q = sqrt(disc);
    const double l = std::max(0.0, floor((-B - q) / (2.0 * A)) - 1.0);
    const double r = std::min((double)N - 1, ceil((-B + q) / (2.0 * A)) + 1.0);
    *lo = (int)l;
    *hi = (int)r;
}

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
            if (c.ypr) vg.any_y = 1; else vg.any_x = 1;
        }
    }
    // Projector tiles, ordered by row tile (a z band of the volume), then
    // view, then column tile, so that the tiles running together on one XCD
    // read one z band.  A tile whose columns mix principal axes, or whose
    // footprint in some chunk exceeds the LDS capacity, falls back to direct
    // gathers.
    std::vector<ConeTile> ty, tx, tf;
    const int nta = (int)cdiv(g.n_u, kTileA), ntb = (int)cdiv(g.n_v, kTileB);
    for (int rt = 0; rt < ntb; ++rt)
        for (int j = 0; j < g.n_views; ++j)
            for (int ct = 0; ct < nta; ++ct) {
                ConeTile t{j, ct * kTileA, rt * kTileB, 1, 0, 1, 0};
                const int a1 = std::min(t.a0 + kTileA, g.n_u) - 1;
                const int b1 = std::min(t.b0 + kTileB, g.n_v) - 1;
                const ConeCol *cj = &cols[(size_t)j * g.n_u];
                bool mixed = false;
                int slo = N, shi = -1, flo = N, fhi = -1;
                for (int a = t.a0; a <= a1; ++a) {
                    const ConeCol &c = cj[a];
                    mixed |= c.ypr != cj[t.a0].ypr;
                    int olo, ohi;
                    valid_slices(c.F0o, c.dFo, N, &olo, &ohi);
                    int clo, chi;
                    fov_slices(c, N, &clo, &chi);
                    for (int b = t.b0; b <= b1; ++b) {
                        int zl, zh;
                        valid_slices(c.Z0 + (long long)b * c.Z1, c.D0 + (long long)b * c.D1, N,
                                     &zl, &zh);
                        const int lo = std::max(olo, zl), hi = std::min(ohi, zh);
                        if (lo > hi) continue;
                        slo = std::min(slo, lo);
                        shi = std::max(shi, hi);
                        const int fl = std::max(lo, clo), fh = std::min(hi, chi);
                        if (fl <= fh) {
                            flo = std::min(flo, fl);
                            fhi = std::max(fhi, fh);
                        }
                    }
                }
                if (slo <= shi) {
                    t.slo = slo;
                    t.shi = shi;
                }
                if (flo <= fhi) {
                    t.flo = flo;
                    t.fhi = fhi;
                }
                bool fits = !mixed;
                if (fits && t.slo <= t.shi) {
                    Corners k;
                    k.init(cj[t.a0], cj[a1], t.b0, b1, (t.slo / kTileS) * kTileS);
                    for (int c0s = (t.slo / kTileS) * kTileS; fits && c0s <= t.shi;
                         c0s += kTileS, k.advance()) {
                        const Footprint f = k.footprint();
                        fits = f.oext <= kFootO && f.zext <= kFootZ;
                    }
                }
                (mixed || !fits ? tf : cj[t.a0].ypr ? ty : tx).push_back(t);
            }
    // adjoint footprints per (view, block of voxel columns)
    const int nbk = (int)cdiv(N, kBpXY);
    std::vector<BpCols> bpc((size_t)g.n_views * nbk * nbk);
    for (int j = 0; j < g.n_views; ++j) {
        const ConeView &vg = views[j];
        const double ax = vg.Sx - vg.Cx, ay = vg.Sy - vg.Cy;
        const double dsd = sqrt(ax * ax + ay * ay), nx = -ax / dsd, ny = -ay / dsd;
        for (int by = 0; by < nbk; ++by)
            for (int bx = 0; bx < nbk; ++bx) {
                double cmin = 1e300, cmax = -1e300, kmin = 1e300, kmax = -1e300;
                for (int q = 0; q < 4; ++q) {
                    const double x = -1.0 + ((q & 1) ? kBpXY * bx + kBpXY + 0.5 : kBpXY * bx - 0.5) * h;
                    const double y = -1.0 + ((q & 2) ? kBpXY * by + kBpXY + 0.5 : kBpXY * by - 0.5) * h;
                    const double Dx = x - vg.Sx, Dy = y - vg.Sy;
                    const double u = (ax * Dy - ay * Dx) / (vg.eux * Dy - vg.euy * Dx);
                    const double col = u / g.du + 0.5 * (double)(g.n_u - 1);
                    const double k = dsd / (Dx * nx + Dy * ny);
                    cmin = std::min(cmin, col);
                    cmax = std::max(cmax, col);
                    kmin = std::min(kmin, k);
                    kmax = std::max(kmax, k);
                }
                BpCols &e = bpc[((size_t)j * nbk + by) * nbk + bx];
                const double lo = std::max(0.0, floor(cmin) - 1.0);
                const double hi = std::min((double)g.n_u - 1, ceil(cmax) + 1.0);
                e.alo = (int)lo;
                e.na = hi >= lo ? (int)(hi - lo) + 1 : 0;
                e.kmin = (float)(kmin * (1.0 - 1e-6));
                e.kmax = (float)(kmax * (1.0 + 1e-6));
            }
    }
    upload(ar, hd->bpcols, bpc);
    hd->zeros.alloc(ar, 64 * sizeof(float));
    zero_fill(ar, hd->zeros);
    // The adjoint stages a footprint per (view, block, z band) when every
    // one fits the caps with two rows to spare (the kernel derives the rows
    // in single precision; its range may differ from this one by a row).
    bool ok = true;
    const double dvinv = 1.0 / g.dv;
    for (size_t e = 0; ok && e < bpc.size(); ++e) {
        ok = bpc[e].na <= kBpA;
        for (int bz = 0; ok && bz < (int)cdiv(N, kZc); ++bz) {
            const double z0 = (double)bz * kZc;
            const double zlo = -1.0 + (z0 - 0.5) * h, zhi = -1.0 + (z0 + kZc + 0.5) * h;
            const double vlo = std::min(zlo * bpc[e].kmin, zlo * bpc[e].kmax);
            const double vhi = std::max(zhi * bpc[e].kmin, zhi * bpc[e].kmax);
            const double blo = std::max(0.0, floor(vlo * dvinv + cv) - 2.0);
            const double bhi = std::min((double)g.n_v - 1, ceil(vhi * dvinv + cv) + 2.0);
            ok = bhi - blo + 1.0 <= kBpB - 2;
        }
    }
    hd->bp_lds = ok;
    // the branch-free walk: rows 1/2 to 1 voxel apart along z everywhere
    // (E1 is linear in the slice: its end slices bound it), and the
    // footprints fit without clamping to the detector
    bool w2 = ok;
    for (size_t e = 0; w2 && e < cols.size(); ++e)
        for (int sx = 0; w2 && sx < 2; ++sx) {
            const long long E1 = cols[e].Z1 + (long long)(sx ? N - 1 : 0) * cols[e].D1;
            w2 = E1 >= (1LL << 39) && E1 < (1LL << 40);
        }
    for (size_t e = 0; w2 && e < bpc.size(); ++e)
        for (int bz = 0; w2 && bz < (int)cdiv(N, kZc); ++bz) {
            const double z0 = (double)bz * kZc;
            const double zlo = -1.0 + (z0 - 0.5) * h, zhi = -1.0 + (z0 + kZc + 0.5) * h;
            const double vlo = std::min(zlo * bpc[e].kmin, zlo * bpc[e].kmax);
            const double vhi = std::max(zhi * bpc[e].kmin, zhi * bpc[e].kmax);
            w2 = (ceil(vhi * dvinv + cv) + 2.0) - (floor(vlo * dvinv + cv) - 2.0) + 1.0 <= kBpB - 2;
        }
    hd->bp_w2 = w2;
    std::vector<ConeTile> all;
    all.reserve(ty.size() + tx.size() + tf.size());
    all.insert(all.end(), ty.begin(), ty.end());
    all.insert(all.end(), tx.begin(), tx.end());
    all.insert(all.end(), tf.begin(), tf.end());
    hd->n_tile_y = (int)ty.size();
    hd->n_tile_x = (int)tx.size();
    hd->n_tile_f = (int)tf.size();
    upload(ar, hd->ccols, cols);
    upload(ar, hd->cviews, views);
    upload(ar, hd->tiles, all);
    // the projector addresses the grid with 32-bit element offsets
    INRCT_REQUIRE((size_t)N * N * N < ((size_t)1 << 31), "cone-beam grid n = %d exceeds 1290",
                  N);
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
// the fraction's upper 32 bits, in units of 2^-32 (fx40_frac's numerator)
__device__ __forceinline__ float fx40_frac32(long long F) { return (float)(unsigned int)(F >> 8); }
__device__ __forceinline__ float fx40_frac(long long F) {
    return fx40_frac32(F) * 2.3283064365386963e-10f;
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

// --------------------------------------------------------------------- P
// z = P u, a tile of kTileA columns x kTileB rows of one view per
// workgroup: lane = column, wave w = rows kRows w .. kRows (w + 1) - 1 of the
// tile, so each thread integrates kRows rays of one column (they share the
// in-plane position and its weight).  Slices are visited in chunks of kTileS: the
// chunk's footprint of u (every tap of every ray of the tile, zero outside
// the grid) is staged in LDS with coalesced loads, then every sample reads
// its four taps from LDS.  A chunk's footprint is small enough (31 KB) for
// four workgroups to share a CU, so some stage while the others integrate.
// Stages the footprint with direct global -> LDS copies (each lane's dword
// lands at the wave's uniform LDS address + 4 lane); lanes whose tap lies
// outside the grid copy a zero.  Consecutive lanes copy consecutive LDS
// dwords: a run of o for y-principal rays, (z, s) pairs for x-principal
// ones.  The copies are waited for at the next barrier.
template <bool YPR>
__device__ __forceinline__ void stage_footprint(float *__restrict__ L, const float *__restrict__ u,
                                                const float *__restrict__ zeros, int N, int s0,
                                                const Footprint &f) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long NN = (long long)N * N;
    const bool inside = f.olo >= 0 && f.olo + f.oext <= N && f.zlo >= 0 && f.zlo + f.zext <= N &&
                        s0 + kTileS <= N;
    if (YPR) {
        // rows (s, z): lane = o; a second pass covers o >= 64, its lanes
        // past the footprint copying nothing (a row holds kLdsZY floats)
        for (int ob = 0; ob < f.oext; ob += 64) {
            if (ob > 0 && ob + lane >= f.oext) break;
            if (inside) {
                // every tap inside the grid: uniform row pointers
                for (int sl = 0; sl < kTileS; ++sl) {
                    const float *row = u + (((long long)(f.zlo + w) * N + s0 + sl) * N + f.olo + ob);
                    for (int z = w; z < f.zext; z += 4, row += 4 * NN)
                        __builtin_amdgcn_global_load_lds(row + lane, L + sl * kLdsSY + z * kLdsZY + ob,
                                                         4, 0, 0);
                }
                continue;
            }
            const int o = f.olo + ob + lane;
            const bool o_in = o >= 0 && o < N;
            for (int sl = 0; sl < kTileS; ++sl) {
                const int sg = s0 + sl;
                const bool so = o_in && sg < N;
                for (int z = w; z < f.zext; z += 4) {
                    const int zg = f.zlo + z;
                    const float *src =
                        so && zg >= 0 && zg < N ? u + (zg * NN + (long long)sg * N + o) : zeros + lane;
                    __builtin_amdgcn_global_load_lds(src, L + sl * kLdsSY + z * kLdsZY + ob, 4, 0, 0);
                }
            }
        }
    } else {
        // rows (o, z): lane = (z offset, s), kZq z rows of kTileS slices per
        // copy; lanes past the footprint's z extent copy nothing
        constexpr int kZq = 64 / kTileS;
        const int sl = lane % kTileS, zq = lane / kTileS;
        if (inside) {
            const long long loff = zq * NN + sl;
            for (int zb = 0; zb < f.zext; zb += kZq) {
                if (zb + zq >= f.zext) break;  // (this lane's z rows are done)
                const float *row = u + (((long long)(f.zlo + zb) * N + f.olo + w) * N + s0) + loff;
                for (int o = w; o < f.oext; o += 4, row += 4 * N)
                    __builtin_amdgcn_global_load_lds(row, L + o * kLdsOX + zb * kLdsZX, 4, 0, 0);
            }
            return;
        }
        const int sg = s0 + sl;
        for (int o = w; o < f.oext; o += 4) {
            const int og = f.olo + o;
            const bool oin = og >= 0 && og < N && sg < N;
            for (int zb = 0; zb < f.zext; zb += kZq) {
                if (zb + zq >= f.zext) break;
                const int zg = f.zlo + zb + zq;
                const float *src = oin && zg >= 0 && zg < N
                                       ? u + (zg * NN + (long long)og * N + sg)
                                       : zeros + lane;
                __builtin_amdgcn_global_load_lds(src, L + o * kLdsOX + zb * kLdsZX, 4, 0, 0);
            }
        }
    }
}

constexpr int kRows = kTileB / 4;  // rays per thread (one column)

template <bool YPR>
__global__ __launch_bounds__(256, 4) void k_cone_fwd_lds(ConeDev g, const ConeTile *__restrict__ tiles,
                                                         int ntiles, const float *__restrict__ u,
                                                         float *__restrict__ zout, int fov_only) {
    __shared__ float L[YPR ? kLdsFloatsY : kLdsFloatsX];
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    if (lb < 0 || lb >= ntiles) return;
    const ConeTile t = tiles[lb];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int a1 = min(t.a0 + kTileA, g.Nu) - 1, b1 = min(t.b0 + kTileB, g.Nv) - 1;
    // lanes past the detector edge follow the last column / row (their
    // positions stay inside the footprint); their results are not written
    const int a = min(t.a0 + lane, a1);
    const ConeCol *cj = g.col + (size_t)t.j * g.Nu;
    const ConeCol c = cj[a];
    const ConeCol ca = cj[t.a0], cb = cj[a1];
    int brow[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) brow[r] = min(t.b0 + kRows * w + r, b1);
    float acc[kRows], acc_d[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) acc[r] = acc_d[r] = 0.f;
    const int lo = fov_only ? t.flo : t.slo, hi = fov_only ? t.fhi : t.shi;
    const int N = g.N;
    const int sfirst = (lo / kTileS) * kTileS;
    // ray positions at the chunk's first slice, relative to the footprint's
    // corner (olo, zlo); corners of the tile for the footprint
    Corners k;
    k.init(ca, cb, t.b0, b1, sfirst);
    long long Fo = c.F0o + (long long)sfirst * c.dFo, Fz[kRows], dFz[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const long long b = brow[r];
        dFz[r] = c.D0 + b * c.D1;
        Fz[r] = c.Z0 + b * c.Z1 + (long long)sfirst * dFz[r];
    }
    int olo = 0, zlo = 0;
    for (int s0 = sfirst; lo <= hi && s0 <= hi; s0 += kTileS, k.advance()) {
        const Footprint f = k.footprint();
        __syncthreads();  // the previous chunk's reads are done
        stage_footprint<YPR>(L, u, g.zeros, N, s0, f);
        // re-base the positions on this chunk's corner
        Fo += (long long)(olo - f.olo) * (1LL << 40);
#pragma unroll
        for (int r = 0; r < kRows; ++r) Fz[r] += (long long)(zlo - f.zlo) * (1LL << 40);
        olo = f.olo;
        zlo = f.zlo;
        __syncthreads();
        // Slice sl's taps are read (into buffer sl & 1) while slice sl - 1
        // is integrated, so the LDS latency overlaps the arithmetic.  The z
        // weight stays the raw fraction (fx40_frac's numerator): a row sums
        // the near taps (acc) and the weighted differences in units of 2^-32
        // (acc_d), joined once at the end.
        constexpr int co = YPR ? 1 : kLdsOX, cz = YPR ? kLdsZY : kLdsZX;
        float v[2][kRows][4], fz[2][kRows], fo[2];
        auto fetch = [&](int sl, int bf) {
            const int io = fx40_int(Fo);
            fo[bf] = fx40_frac(Fo);
            const float *Ls = L + (YPR ? sl * kLdsSY + io : sl + io * kLdsOX);
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const float *p = Ls + fx40_int(Fz[r]) * cz;
                v[bf][r][0] = p[0];
                v[bf][r][1] = p[co];
                v[bf][r][2] = p[cz];
                v[bf][r][3] = p[cz + co];
                fz[bf][r] = fx40_frac32(Fz[r]);
                Fz[r] += dFz[r];
            }
            Fo += c.dFo;
        };
        fetch(0, 0);
#pragma unroll
        for (int sl = 0; sl < kTileS; ++sl) {
            if (sl + 1 < kTileS) fetch(sl + 1, (sl + 1) & 1);
            __builtin_amdgcn_sched_barrier(0);
            const int bf = sl & 1;
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const float t0 = fmaf(fo[bf], v[bf][r][1] - v[bf][r][0], v[bf][r][0]);
                const float t1 = fmaf(fo[bf], v[bf][r][3] - v[bf][r][2], v[bf][r][2]);
                acc[r] += t0;
                acc_d[r] = fmaf(fz[bf][r], t1 - t0, acc_d[r]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (t.a0 + lane > a1) return;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int b = t.b0 + kRows * w + r;
        const float sum = fmaf(acc_d[r], 2.3283064365386963e-10f, acc[r]);
        if (b <= b1) zout[((size_t)t.j * g.Nv + b) * g.Nu + a] = sum * cone_step(g, c, b);
    }
}

// The same tile by direct gathers from u with bounds tests, for tiles whose
// columns mix principal axes or whose footprint exceeds the LDS capacity.
__global__ __launch_bounds__(256) void k_cone_fwd_direct(ConeDev g,
                                                         const ConeTile *__restrict__ tiles,
                                                         int ntiles, const float *__restrict__ u,
                                                         float *__restrict__ zout) {
    if ((int)blockIdx.x >= ntiles) return;
    const ConeTile t = tiles[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int a = t.a0 + lane;
    if (a >= g.Nu) return;
    const ConeCol c = g.col[(size_t)t.j * g.Nu + a];
    const int N = g.N;
    const long long NN = (long long)N * N;
    auto at = [&](int iz, int is, int io) -> float {
        if (iz < 0 || iz >= N || io < 0 || io >= N) return 0.f;
        return c.ypr ? u[iz * NN + (long long)is * N + io] : u[iz * NN + (long long)io * N + is];
    };
    for (int r = 0; r < kRows; ++r) {
        const int b = t.b0 + kRows * w + r;
        if (b >= g.Nv) break;
        const long long F0z = c.Z0 + (long long)b * c.Z1, dFz = c.D0 + (long long)b * c.D1;
        int lo1, hi1, lo2, hi2;
        range40_exact(c.F0o, c.dFo, N, &lo1, &hi1);
        range40_exact(F0z, dFz, N, &lo2, &hi2);
        float acc = 0.f;
        for (int s = max(lo1, lo2); s <= min(hi1, hi2); ++s) {
            const long long Fo = c.F0o + (long long)s * c.dFo, Fz = F0z + (long long)s * dFz;
            const int io = fx40_int(Fo), iz = fx40_int(Fz);
            const float fo = fx40_frac(Fo), fz = fx40_frac(Fz);
            const float t0 = fmaf(fo, at(iz, s, io + 1) - at(iz, s, io), at(iz, s, io));
            const float t1 =
                fmaf(fo, at(iz + 1, s, io + 1) - at(iz + 1, s, io), at(iz + 1, s, io));
            acc += fmaf(fz, t1 - t0, t0);
        }
        zout[((size_t)t.j * g.Nv + b) * g.Nu + a] = acc * cone_step(g, c, b);
    }
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
    const float a1 = fmaf(u1, g.inv_du, c), a2 = fmaf(u2, g.inv_du, c);
    // the columns inside [a1, a2], widened by the margin
    float l = ceilf(fminf(a1, a2) - 0.01f), r = floorf(fmaxf(a1, a2) + 0.01f);
    l = fmaxf(l, 0.f);
    r = fminf(r, (float)(g.Nu - 1));
    *lo = (int)l;
    *hi = (int)r;
}

// (P^T r) of view j for voxels (ix, iy, z0 .. z0 + ZC - 1), accumulated
// into acc.  The step-weighted residual of the view is read as R[(b - blo)
// rstride + (a - alo)] for detector rows [blo, bhi] and columns [alo, ahi],
// and column a's record as C[a - alo]; both may be staged copies in LDS or
// the arrays themselves.  Every voxel receives its terms in increasing row
// order, whatever the source.
template <int ZC>
__device__ __forceinline__ void cone_gather_view(const ConeDev &g, const ConeView &vg,
                                                 const float *__restrict__ R, int rstride,
                                                 const ConeCol *__restrict__ C, int alo, int ahi,
                                                 int blo, int bhi, int ix, int iy, int z0,
                                                 float (&acc)[ZC]) {
    const float h = (float)g.h;
    const float x = (float)(-1.0 + (ix + 0.5) * g.h), y = (float)(-1.0 + (iy + 0.5) * g.h);
    for (int pass = 0; pass < 2; ++pass) {
        const bool ypass = pass == 0;
        if (ypass ? !vg.any_y : !vg.any_x) continue;
        const int s = ypass ? iy : ix, o = ypass ? ix : iy;
        int lo, hi;
        if (ypass) cone_cols(g, vg, x - h, y, x + h, y, &lo, &hi);
        else cone_cols(g, vg, x, y - h, x, y + h, &lo, &hi);
        lo = max(lo, alo);
        hi = min(hi, ahi);
        for (int a = lo; a <= hi; ++a) {
            const ConeCol c = C[a - alo];
            if ((c.ypr != 0) != ypass) continue;
            const long long Fo = c.F0o + (long long)s * c.dFo;
            const int io = fx40_int(Fo);
            if (io != o && io != o - 1) continue;
            const float fo = fx40_frac(Fo);
            const float wo = io == o ? 1.f - fo : fo;
            const long long E0 = c.Z0 + (long long)s * c.D0;
            const long long E1 = c.Z1 + (long long)s * c.D1;  // > 0
            // first row whose stencil reaches z0 - 1
            const long long lo_t = (long long)(z0 - 1) * (1LL << 40);
            // row estimate in single precision; the walks below make it exact
            float bd = floorf((float)(lo_t - E0) * __builtin_amdgcn_rcpf((float)E1)) - 1.f;
            bd = bd < (float)blo ? (float)blo : (bd > (float)(bhi + 1) ? (float)(bhi + 1) : bd);
            int b = (int)bd;
            long long ph = E0 + (long long)b * E1;
            while (b > blo && ph - E1 >= lo_t) {
                --b;
                ph -= E1;
            }
            while (b <= bhi && ph < lo_t) {
                ++b;
                ph += E1;
            }
            // One pass over the rows from b on: a row whose stencil starts
            // at voxel i0 gives (1 - w) to i0 and w to i0 + 1.
            int ri = (b - blo) * rstride + (a - alo);
            while (b <= bhi && fx40_int(ph) == z0 - 1) {
                acc[0] += wo * fx40_frac(ph) * R[ri];
                ++b;
                ph += E1;
                ri += rstride;
            }
#pragma unroll
            for (int jz = 0; jz < ZC; ++jz) {
                while (b <= bhi && fx40_int(ph) == z0 + jz) {
                    const float w = fx40_frac(ph);
                    const float r = R[ri];
                    acc[jz] += wo * (1.f - w) * r;
                    if (jz + 1 < ZC) acc[jz + 1] += wo * w * r;
                    ++b;
                    ph += E1;
                    ri += rstride;
                }
            }
        }
    }
}

// cone_gather_view for geometries whose detector rows are between half a
// voxel and one voxel apart along z at every column and slice (E1 in
// [1/2, 1)): every voxel band [z, z + 1) then holds one or two rows, so the
// walk visits, for each band, the band's first row and the row after it
// (used only when it lies in the band), with no data-dependent branch.  R
// must hold every row whose stencil reaches the segment, zeros for rows off
// the detector, and one more row (the walk reads a row past the last).
// One column's contribution to voxels (o, s, z0 .. z0 + ZC - 1) under the
// walk below: acc[jz] += wo_s 2^32 (sum over its rows of the row's z weight
// for voxel z0 + jz times the residual), for a column record c at slice s,
// with rows read from R (row stride rstride, this column's entries starting
// at R + (b - blo) rstride).  Rows must lie between half a voxel and one
// voxel apart along z (E1 in [1/2, 1)): every voxel band [z, z + 1) then
// holds one or two rows, so the walk visits, for each band, the band's first
// row and the row after it (used only when it lies in the band), with no
// data-dependent branch.  R must hold every row whose stencil reaches the
// segment, zeros for rows off the detector, and one more row (the walk
// reads a row past the last).
template <int ZC>
__device__ __forceinline__ void w2_column(const float *__restrict__ R, int rstride,
                                          const ConeCol &c, int s, int a_local, int blo, int z0,
                                          float wo_s, float (&acc)[ZC]) {
    const long long E0 = c.Z0 + (long long)s * c.D0;
    const long long E1 = c.Z1 + (long long)s * c.D1;
    // the first row whose stencil reaches z0 - 1: an estimate from the high
    // bits (E1 >= 2^39, so E1 >> 24 keeps 16 bits and the estimate is within
    // a tenth of a row), then exact
    const long long lo_t = (long long)(z0 - 1) * (1LL << 40);
    int b = (int)floorf((float)(int)((lo_t - E0) >> 24) *
                        __builtin_amdgcn_rcpf((float)(int)(E1 >> 24)));
    long long ph = E0 + (long long)b * E1;
    if (ph >= lo_t) {
        --b;
        ph -= E1;
    }
    if (ph < lo_t) {
        ++b;
        ph += E1;
    }
    if (ph < lo_t) {
        ++b;
        ph += E1;
    }
    const float *rp = R + (b - blo) * rstride + a_local;
    // band jz = -1 .. ZC - 1: rows with floor(phi) = z0 + jz give (1 - w) to
    // voxel jz and w to voxel jz + 1.  The weights stay in units of 2^-32: w
    // is fx40_frac's numerator; the power of two is in wo_s.  Positions are
    // taken relative to voxel z0 (the fractions are unchanged): row A of band
    // jz lies in band jz and row B in band jz or jz + 1 (rows are 1/2 to 1
    // voxel apart), so one compare of B's high word with (jz + 1) << 8 tells
    // which.
    ph -= (long long)z0 << 40;
    // both rows of a band are read unconditionally (R holds the row after
    // the last), so a band is straight-line code; the next band's rows are
    // read before this band's arithmetic (their place depends on positions
    // only), so the LDS latency overlaps it
    float rA = rp[0], rB0 = rp[rstride];
#pragma unroll
    for (int jz = -1; jz < ZC; ++jz) {
        const long long phB = ph + E1;
        const bool inB = (int)(phB >> 32) < (jz + 1) * 256;
        rp += inB ? 2 * rstride : rstride;
        float nA = 0.f, nB0 = 0.f;
        if (jz + 1 < ZC) {
            nA = rp[0];
            nB0 = rp[rstride];
        }
        // keep the reads above this band's arithmetic
        __builtin_amdgcn_sched_barrier(0);
        const float rB = inB ? rB0 : 0.f;
        const float cA = fx40_frac32(ph), cB = fx40_frac32(phB);
        const float q = fmaf(cB, rB, cA * rA);
        // the lower voxel's share (2^32 - cA) rA + (2^32 - cB) rB, formed as
        // 2^32 (rA + rB) - q: its rounding is within 2^-24 of the band's
        // full-weight term
        const float qn = fmaf(4294967296.f, rA + rB, -q);
        if (jz >= 0) acc[jz] = fmaf(qn, wo_s, acc[jz]);
        if (jz + 1 < ZC) acc[jz + 1] = fmaf(q, wo_s, acc[jz + 1]);
        ph = inB ? phB + E1 : phB;
        rA = nA;
        rB0 = nB0;
    }
}

// cone_gather_view for geometries whose detector rows are between half a
// voxel and one voxel apart along z at every column and slice (w2_column).
template <int ZC>
__device__ __forceinline__ void cone_gather_view_w2(const ConeDev &g, const ConeView &vg,
                                                    const float *__restrict__ R, int rstride,
                                                    const ConeCol *__restrict__ C, int alo, int ahi,
                                                    int blo, int ix, int iy, int z0,
                                                    float (&acc)[ZC]) {
    const float h = (float)g.h;
    const float x = (float)(-1.0 + (ix + 0.5) * g.h), y = (float)(-1.0 + (iy + 0.5) * g.h);
    for (int pass = 0; pass < 2; ++pass) {
        const bool ypass = pass == 0;
        if (ypass ? !vg.any_y : !vg.any_x) continue;
        const int s = ypass ? iy : ix, o = ypass ? ix : iy;
        int lo, hi;
        if (ypass) cone_cols(g, vg, x - h, y, x + h, y, &lo, &hi);
        else cone_cols(g, vg, x, y - h, x, y + h, &lo, &hi);
        lo = max(lo, alo);
        hi = min(hi, ahi);
        for (int a = lo; a <= hi; ++a) {
            const ConeCol c = C[a - alo];
            if ((c.ypr != 0) != ypass) continue;
            const long long Fo = c.F0o + (long long)s * c.dFo;
            const int io = fx40_int(Fo);
            if (io != o && io != o - 1) continue;
            const float fo = fx40_frac(Fo);
            const float wo = io == o ? 1.f - fo : fo;
            w2_column<ZC>(R, rstride, c, s, a - alo, blo, z0, wo * 2.3283064365386963e-10f, acc);
        }
    }
}

// (P^T r) for voxels (ix, iy, z0 .. z0 + ZC - 1) over all views, reading the
// residual and the column records in place.
template <int ZC>
__device__ __forceinline__ void cone_gather(const ConeDev &g, const float *__restrict__ rs,
                                            int ix, int iy, int z0, float (&acc)[ZC]) {
    for (int j = 0; j < g.V; ++j)
        cone_gather_view<ZC>(g, g.view[j], rs + (size_t)j * g.Nv * g.Nu, g.Nu,
                             g.col + (size_t)j * g.Nu, 0, g.Nu - 1, 0, g.Nv - 1, ix, iy, z0, acc);
}


struct BpFoot {
    int alo, na, blo, nb;
};

// Detector footprint of view j for the block (bx, by) and the z band
// [z0, z0 + kZc): the block's columns, and the rows whose stencil reaches
// z in [z0 - 1, z0 + kZc] (world z from the band, times D_sd / d), with two
// rows of margin.
template <bool W2>
__device__ __forceinline__ BpFoot bp_foot(const ConeDev &g, int j, int nbk, int bx, int by,
                                          int z0) {
    const BpCols e = g.bpc[((size_t)j * nbk + by) * nbk + bx];
    const float h = (float)g.h;
    const float zlo = -1.f + ((float)z0 - 0.5f) * h, zhi = -1.f + ((float)z0 + kZc + 0.5f) * h;
    const float vlo = fminf(zlo * e.kmin, zlo * e.kmax), vhi = fmaxf(zhi * e.kmin, zhi * e.kmax);
    const float inv = 1.f / g.dvf;
    // the branch-free walk reads rows off the detector too (staged as zeros)
    int blo = (int)floorf(vlo * inv + g.cvf) - 2, bhi = (int)ceilf(vhi * inv + g.cvf) + 2;
    if (!W2) {
        blo = max(0, blo);
        bhi = min(g.Nv - 1, bhi);
    }
    BpFoot f;
    f.alo = e.alo;
    f.na = min(e.na, kBpA);
    f.blo = blo;
    // (the host checked that every footprint fits with two rows to spare;
    // the clamp only guards the staging buffer)
    f.nb = min(bhi >= blo ? bhi - blo + 1 : 0, kBpB);
    return f;
}

// v = P^T r on the full grid.  A block is 16 x 16 voxel columns (a wave an
// 8 x 8 patch) by kZc voxels along z, one thread per column segment.  View
// by view, the block's detector footprint of the step-weighted residual and
// the footprint's column records are staged in LDS (the next view's values
// are loaded into registers while the current view is gathered), so the
// row walks read LDS.  Used when every footprint fits the caps (checked when
// the geometry is built).  Gather only: no atomics.
template <bool W2>
__global__ __launch_bounds__(256) void k_cone_bp_lds(ConeDev g, const float *__restrict__ rs,
                                                     float *__restrict__ v, int nbk) {
    __shared__ float R[2][(kBpB + 1) * kBpRs];
    __shared__ ConeCol C[2][kBpA];
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    if (lb < 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int bx = lb % nbk, by = (lb / nbk) % nbk, bz = lb / (nbk * nbk);
    const int ix = bx * kBpXY + (wave & 1) * 8 + (lane & 7);
    const int iy = by * kBpXY + (wave >> 1) * 8 + (lane >> 3);
    const int z0 = bz * kZc;
    const bool active = ix < g.N && iy < g.N;
    float acc[kZc];
#pragma unroll
    for (int i = 0; i < kZc; ++i) acc[i] = 0.f;
    // staging: thread t holds detector column alo + (t & 63) of rows
    // blo + (t >> 6) + 4 q, and dwords (t & 15) + 16 q' of the records
    constexpr int kRq = kBpB / 4, kCw = (int)(sizeof(ConeCol) / 4);
    constexpr int kCq = kBpA * kCw / 256;
    float rv[kRq];
    int cv[kCq];
    auto load = [&](int j, const BpFoot &f) {
        const float *rj = rs + (size_t)j * g.Nv * g.Nu;
        const int col = threadIdx.x & 63;
#pragma unroll
        for (int q = 0; q < kRq; ++q) {
            const int row = (threadIdx.x >> 6) + 4 * q;
            const int b = f.blo + row;
            rv[q] = col < f.na && row < f.nb && b >= 0 && b < g.Nv
                        ? rj[(size_t)b * g.Nu + f.alo + col]
                        : 0.f;
        }
        const int *cj = (const int *)(g.col + (size_t)j * g.Nu + f.alo);
#pragma unroll
        for (int q = 0; q < kCq; ++q) {
            const int w = threadIdx.x + 256 * q;
            cv[q] = w < f.na * kCw ? cj[w] : 0;
        }
    };
    auto store = [&](int buf, const BpFoot &f) {
        const int col = threadIdx.x & 63;
#pragma unroll
        for (int q = 0; q < kRq; ++q) R[buf][((threadIdx.x >> 6) + 4 * q) * kBpRs + col] = rv[q];
        int *cw = (int *)C[buf];
#pragma unroll
        for (int q = 0; q < kCq; ++q) cw[threadIdx.x + 256 * q] = cv[q];
    };
    BpFoot f = bp_foot<W2>(g, 0, nbk, bx, by, z0);
    load(0, f);
    store(0, f);
    __syncthreads();
    for (int j = 0; j < g.V; ++j) {
        const int buf = j & 1;
        BpFoot fn;
        if (j + 1 < g.V) {
            fn = bp_foot<W2>(g, j + 1, nbk, bx, by, z0);
            load(j + 1, fn);
        }
        if (active && f.na > 0 && f.nb > 0) {
            if (W2)
                cone_gather_view_w2<kZc>(g, g.view[j], R[buf], kBpRs, C[buf], f.alo,
                                         f.alo + f.na - 1, f.blo, ix, iy, z0, acc);
            else
                cone_gather_view<kZc>(g, g.view[j], R[buf], kBpRs, C[buf], f.alo, f.alo + f.na - 1,
                                      f.blo, f.blo + f.nb - 1, ix, iy, z0, acc);
        }
        if (j + 1 < g.V) {
            store(buf ^ 1, fn);
            f = fn;
        }
        __syncthreads();
    }
    if (!active) return;
    const size_t NN = (size_t)g.N * g.N;
#pragma unroll
    for (int i = 0; i < kZc; ++i)
        if (z0 + i < g.N) v[(size_t)(z0 + i) * NN + (size_t)iy * g.N + ix] = acc[i];
}

// v = P^T r reading the residual in place, for geometries whose footprints
// exceed the LDS caps.
__global__ __launch_bounds__(256) void k_cone_bp_direct(ConeDev g, const float *__restrict__ rs,
                                                        float *__restrict__ v, int nbk) {
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    if (lb < 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int bx = lb % nbk, by = (lb / nbk) % nbk, bz = lb / (nbk * nbk);
    const int ix = bx * kBpXY + (wave & 1) * 8 + (lane & 7);
    const int iy = by * kBpXY + (wave >> 1) * 8 + (lane >> 3);
    const int z0 = bz * kZc;
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
void cone_project(inrct_geom *hd, const float *u, float *z, bool fov_only, hipStream_t s,
                  const float *ut) {
    const ConeDev d = hd->cone();
    const ConeTile *t = hd->tiles.as<ConeTile>();
    if (hd->n_tile_y > 0) {
        hipLaunchKernelGGL(k_cone_fwd_lds<true>, dim3((unsigned)hd->n_tile_y), dim3(256), 0, s, d,
                           t, hd->n_tile_y, u, z, fov_only ? 1 : 0);
        INRCT_CHECK_LAUNCH();
    }
    if (hd->n_tile_x > 0) {
        // with ut ([z][x][y]) an x-principal ray's slices are rows, as a
        // y-principal ray's are in u: the same kernel and footprints apply
        if (ut)
            hipLaunchKernelGGL(k_cone_fwd_lds<true>, dim3((unsigned)hd->n_tile_x), dim3(256), 0,
                               s, d, t + hd->n_tile_y, hd->n_tile_x, ut, z, fov_only ? 1 : 0);
        else
            hipLaunchKernelGGL(k_cone_fwd_lds<false>, dim3((unsigned)hd->n_tile_x), dim3(256), 0,
                               s, d, t + hd->n_tile_y, hd->n_tile_x, u, z, fov_only ? 1 : 0);
        INRCT_CHECK_LAUNCH();
    }
    if (hd->n_tile_f > 0) {
        hipLaunchKernelGGL(k_cone_fwd_direct, dim3((unsigned)hd->n_tile_f), dim3(256), 0, s, d,
                           t + hd->n_tile_y + hd->n_tile_x, hd->n_tile_f, u, z);
        INRCT_CHECK_LAUNCH();
    }
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
    const int nbk = (int)cdiv(d.N, kBpXY), nbz = (int)cdiv(d.N, kZc);
    if (hd->bp_lds && hd->bp_w2)
        hipLaunchKernelGGL(k_cone_bp_lds<true>, dim3((unsigned)(nbk * nbk * nbz)), dim3(256), 0, s,
                           d, rs, v, nbk);
    else if (hd->bp_lds)
        hipLaunchKernelGGL(k_cone_bp_lds<false>, dim3((unsigned)(nbk * nbk * nbz)), dim3(256), 0, s,
                           d, rs, v, nbk);
    else
        hipLaunchKernelGGL(k_cone_bp_direct, dim3((unsigned)(nbk * nbk * nbz)), dim3(256), 0, s, d,
                           rs, v, nbk);
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
