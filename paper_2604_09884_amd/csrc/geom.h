// Internal geometry handle shared by the projector sources.
#pragma once

#include "common.h"

namespace inrct {

// 2D parallel and fan beam: one record per (view, detector bin).  The
// interpolation position of the ray's non-principal coordinate at slice s
// is the exact 32.32 fixed-point integer F0 + s dF, in P and in P^T.
struct Col2D {
    long long F0, dF;
};

// Per view, in single precision, what the adjoint needs to find the
// candidate bins of a pixel: parallel beam uses the detector axis (eux,
// euy); fan beam the source S, S - C and the detector axis.  Bins are split
// by principal axis: [0, ysplit) are y-principal iff yfirst, [ysplit, Nu)
// the other way (a fan narrower than 90 degrees has at most one change).
struct View2D {
    float sx, sy, ax, ay, eux, euy;
    int ysplit, yfirst;
};

struct GeomDev {
    int kind, N, V, Nu, Nv;
    double h, du, dv;
    const Col2D *col;    // [V][Nu]
    const float *step;   // [V][Nu] slice step length h |d| / |d_axis|
    const View2D *view;  // [V]
};

// 3D cone beam: one record per (view, detector column), 24.40 fixed point.
// The interpolation positions of ray (column a, row b) at slice s are
//   phi_other(s)  = F0o + s dFo
//   phi_z(s, b)   = Z0 + s D0 + b (Z1 + s D1)
// (exact integer arithmetic; the z position is affine in the detector row
// because the row axis is the z axis).
struct ConeCol {
    long long F0o, dFo, Z0, D0, Z1, D1;
    float dxy2;   // squared in-plane length of the ray direction
    float dz0;    // z component of the direction before the row offset
    float hinv;   // h / |d_axis|
    int ypr;      // 1: y is the principal axis
};

struct ConeView {
    double Sx, Sy, Cx, Cy, eux, euy;
    int any_y, any_x;
};

// A tile of the LDS-staged cone projector: rays of view j, detector
// columns [a0, a0 + kTileA) and rows [b0, b0 + kTileB) (clipped to the
// detector), all with one principal axis.  Slices are visited in chunks of
// kTileS aligned to multiples of kTileS; [slo, shi] holds every slice where
// some ray of the tile has a tap inside the grid, [flo, fhi] (a sub-range)
// every slice where some ray passes the FOV cylinder (all a projection of
// an image that vanishes outside the FOV needs).  An empty range has
// lo > hi.
constexpr int kTileA = 64, kTileB = 24, kTileS = 4;
struct ConeTile {
    int j, a0, b0;
    int slo, shi, flo, fhi;
};

// The adjoint works on blocks of kBpXY x kBpXY voxel columns.  For each
// view and block: the detector columns [alo, alo + na) whose rays can touch
// the block's voxels (central projection of the block's in-plane box widened
// by one voxel, plus one column of margin), and the extremes of D_sd / d
// over the box, d the depth along the view's central ray, from which the
// rows touching a z band follow (row coordinate = z D_sd / d).
constexpr int kBpXY = 16;
struct BpCols {
    int alo, na;
    float kmin, kmax;
};

struct ConeDev {
    int N, V, Nu, Nv;
    double h, du;
    float inv_du;          // 1 / du
    float dvf, cvf;        // row pitch and (Nv - 1)/2
    const ConeCol *col;    // [V][Nu]
    const ConeView *view;  // [V]
    const BpCols *bpc;     // [V][nb][nb], nb = ceil(N / kBpXY)
    const float *zeros;    // 64 zero floats (the source of staged taps outside the grid)
};

}  // namespace inrct

struct inrct_geom {
    inrct::Workspace ws;
    ct_geometry g;
    int N = 0, dim = 0;
    std::vector<double> angles;
    inrct::DevBuf cols, steps, views, q, partials;
    int n_partials = 0;
    // cone beam: per-column records, per-view records, and the projector's
    // tile lists (LDS-staged tiles by principal axis, then the tiles that
    // fall back to direct gathers)
    inrct::DevBuf ccols, cviews, tiles, bpcols, zeros;
    // 2D: transposed copy of the image for the x-principal rays
    inrct::DevBuf ut;
    int n_tile_y = 0, n_tile_x = 0, n_tile_f = 0;
    bool bp_lds = false;  // every adjoint footprint fits the LDS caps
    bool bp_w2 = false;   // and rows lie 1/2 to 1 voxel apart: the branch-free walk
    inrct::GeomDev dev() const {
        inrct::GeomDev d;
        d.kind = g.kind;
        d.N = N;
        d.V = g.n_views;
        d.Nu = g.n_u;
        d.Nv = g.n_v;
        d.h = 2.0 / N;
        d.du = g.du;
        d.dv = g.dv;
        d.col = cols.as<inrct::Col2D>();
        d.step = steps.as<float>();
        d.view = views.as<inrct::View2D>();
        return d;
    }
    inrct::ConeDev cone() const {
        inrct::ConeDev d;
        d.N = N;
        d.V = g.n_views;
        d.Nu = g.n_u;
        d.Nv = g.n_v;
        d.h = 2.0 / N;
        d.du = g.du;
        d.inv_du = (float)(1.0 / g.du);
        d.dvf = (float)g.dv;
        d.cvf = 0.5f * (float)(g.n_v - 1);
        d.col = ccols.as<inrct::ConeCol>();
        d.view = cviews.as<inrct::ConeView>();
        d.bpc = bpcols.as<inrct::BpCols>();
        d.zeros = zeros.as<float>();
        return d;
    }
    int64_t m() const { return (int64_t)g.n_views * g.n_v * g.n_u; }
};

namespace inrct {
void cone_build(inrct_geom *h, Arena &a);
void check_geom_args(const ct_geometry *g, const inr_grid *grid);
inrct_geom *fresh_geom(const ct_geometry *g, const inr_grid *grid);
void build_geom(inrct_geom *h, Arena &ar);
void cone_project(inrct_geom *h, const float *u, float *z, bool fov_only, hipStream_t s,
                  const float *ut = nullptr);
// z = P u; with fov_only the caller guarantees u = 0 outside the FOV (the
// projector may then skip slices that lie outside it).
// z = P u.  For a cone geometry, ut (optional) is u transposed in every xy
// plane ([z][x][y]); given it, x-principal rays read it with the y-principal
// kernel (rows along their own axis) instead of staging columns of u.
void project(inrct_geom *geom, const float *u, float *z, hipStream_t s, bool fov_only = false,
             const float *ut = nullptr);
// ut = u transposed in each of `planes` N x N planes
void transpose_planes(const float *u, float *ut, int N, int planes, hipStream_t s);
// a cone geometry whose projector has x-principal tiles (those read ut)
inline bool geom_reads_transpose(const inrct_geom *g) {
    return g->g.kind == INRCT_CONE3D && g->n_tile_x > 0;
}
void cone_backproject(inrct_geom *h, const float *r, float *v, hipStream_t s);
void cone_backproject_at(inrct_geom *h, const float *r, const int32_t *idx, int64_t k,
                         float *out, hipStream_t s);
}  // namespace inrct
