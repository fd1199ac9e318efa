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

struct ConeDev {
    int N, V, Nu, Nv;
    double h, du;
    float dvf, cvf;        // row pitch and (Nv - 1)/2
    const ConeCol *col;    // [V][Nu]
    const ConeView *view;  // [V]
};

}  // namespace inrct

struct inrct_geom {
    inrct::Workspace ws;
    ct_geometry g;
    int N = 0, dim = 0;
    std::vector<double> angles;
    inrct::DevBuf cols, steps, views, q, partials;
    int n_partials = 0;
    // cone beam
    inrct::DevBuf ccols, cviews, ut;
    bool any_x = false;
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
        d.dvf = (float)g.dv;
        d.cvf = 0.5f * (float)(g.n_v - 1);
        d.col = ccols.as<inrct::ConeCol>();
        d.view = cviews.as<inrct::ConeView>();
        return d;
    }
    int64_t m() const { return (int64_t)g.n_views * g.n_v * g.n_u; }
};

namespace inrct {
void cone_build(inrct_geom *h, Arena &a);
void check_geom_args(const ct_geometry *g, const inr_grid *grid);
inrct_geom *fresh_geom(const ct_geometry *g, const inr_grid *grid);
void build_geom(inrct_geom *h, Arena &ar);
void cone_project(inrct_geom *h, const float *u, float *z, hipStream_t s);
void cone_backproject(inrct_geom *h, const float *r, float *v, hipStream_t s);
void cone_backproject_at(inrct_geom *h, const float *r, const int32_t *idx, int64_t k,
                         float *out, hipStream_t s);
}  // namespace inrct
