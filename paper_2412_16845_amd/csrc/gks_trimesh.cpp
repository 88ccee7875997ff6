// Triangle-mesh ingest: topology checks and the per-cell face geometry the triangle kernels read.
//
// Every cell owns its three faces in the kernels (each face is evaluated by both of its cells,
// each from its own side with its own outward normal: the flux of a face seen from the other
// side is the negative, which the lattice's half-turn symmetry guarantees), so the geometry is
// stored per cell and face slot (layout in gks_internal.h):
//   nb     neighbour cell, or -(1 + bc) on a boundary face (non-reflecting or PEC)
//   n      outward unit normal
//   lw     |l_s| / |Omega_i|
//   a      x_s - x_i   (face midpoint minus the cell centroid: the cell's reconstruction), slots
//          0 and 1 only: the offsets of the three midpoints from the centroid add to zero
//   b      x_s - x_nb  (the same for the neighbour; 0 on boundary faces)
//   W      gradient weights, grad U_i = sum_k W_k (U_k - U_i) over the neighbours or boundary
//          ghosts: Green-Gauss (n |l| / (2 |Omega|)) or the least-squares fit (M^-1 d_k, with
//          d_k the neighbour's centroid, or the centroid's mirror image across a boundary face,
//          minus x_i, and M = sum_k d_k d_k^T)
// Everything is computed in double precision (Sec. 3.1: Green-Gauss gradients, reconstruction
// at the face midpoint).
#include <cmath>
#include <cstdio>
#include <vector>

#include "gks_internal.h"

namespace gks {

bool build_tri_geometry(const gks_mesh_desc *m, int gradient, TriGeometry &g, char *err, size_t errlen)
{
    const int64_t nv = m->nverts, nc = m->ncells, nf = m->nfaces;
    if (nv < 3 || nc < 1 || nf < 3) {
        std::snprintf(err, errlen, "a triangle mesh needs >= 3 vertices, >= 1 cell and >= 3 faces");
        return false;
    }
    if (nc > (int64_t)0x3FFFFFFF || nf > (int64_t)0x7FFFFFFF || nv > (int64_t)0x7FFFFFFF) {
        std::snprintf(err, errlen, "mesh too large for 32-bit indexing");
        return false;
    }
    if (!m->vert_xy || !m->cell_verts || !m->face_cells || !m->face_verts) {
        std::snprintf(err, errlen, "vert_xy, cell_verts, face_cells and face_verts are required");
        return false;
    }
    for (int64_t v = 0; v < 2 * nv; ++v)
        if (!std::isfinite(m->vert_xy[v])) {
            std::snprintf(err, errlen, "vertex %lld is not finite", (long long)(v / 2));
            return false;
        }
    std::vector<double> cx(nc), cy(nc), area(nc);
    for (int64_t c = 0; c < nc; ++c) {
        const int32_t *t = m->cell_verts + 3 * c;
        for (int k = 0; k < 3; ++k)
            if (t[k] < 0 || t[k] >= nv) {
                std::snprintf(err, errlen, "cell %lld has vertex %d outside [0, %lld)", (long long)c, t[k], (long long)nv);
                return false;
            }
        const double *p0 = m->vert_xy + 2 * t[0], *p1 = m->vert_xy + 2 * t[1], *p2 = m->vert_xy + 2 * t[2];
        const double a2 = (p1[0] - p0[0]) * (p2[1] - p0[1]) - (p1[1] - p0[1]) * (p2[0] - p0[0]);
        area[c] = 0.5 * std::fabs(a2);
        if (!(area[c] > 0)) {
            std::snprintf(err, errlen, "cell %lld is degenerate", (long long)c);
            return false;
        }
        cx[c] = (p0[0] + p1[0] + p2[0]) / 3.0;
        cy[c] = (p0[1] + p1[1] + p2[1]) / 3.0;
    }
    auto has_vertex = [&](int64_t c, int32_t v) {
        const int32_t *t = m->cell_verts + 3 * c;
        return t[0] == v || t[1] == v || t[2] == v;
    };
    std::vector<int32_t> count(nc, 0);
    g.ncell = nc;
    g.nb.assign(3 * nc, 0);
    g.geo.assign((size_t)TRI_GEO_ROWS * nc, 0.0);
    std::vector<double> perim(nc, 0.0);
    std::vector<double> am((size_t)6 * nc, 0.0);   // x_s - x_i of every slot: [slot][x|y][cell]
    auto G = [&](int row, int64_t c) -> double & { return g.geo[(size_t)row * nc + c]; };
    for (int64_t s = 0; s < nf; ++s) {
        const int32_t L = m->face_cells[2 * s], R = m->face_cells[2 * s + 1];
        const int32_t v0 = m->face_verts[2 * s], v1 = m->face_verts[2 * s + 1];
        if (L < 0 || L >= nc) {
            std::snprintf(err, errlen, "face %lld: owner %d outside [0, %lld)", (long long)s, L, (long long)nc);
            return false;
        }
        if (R >= nc || R == L || (R < 0 && R != -(1 + GKS_BC_NONREFLECT) && R != -(1 + GKS_BC_PEC))) {
            std::snprintf(err, errlen, "face %lld: neighbour %d is neither a cell other than the owner nor a "
                                       "non-reflecting (-2) or PEC (-3) boundary", (long long)s, R);
            return false;
        }
        if (v0 < 0 || v0 >= nv || v1 < 0 || v1 >= nv || v0 == v1 || !has_vertex(L, v0) || !has_vertex(L, v1) ||
            (R >= 0 && (!has_vertex(R, v0) || !has_vertex(R, v1)))) {
            std::snprintf(err, errlen, "face %lld: its vertices are not an edge of its cells", (long long)s);
            return false;
        }
        const double *p = m->vert_xy + 2 * v0, *q = m->vert_xy + 2 * v1;
        const double mx = 0.5 * (p[0] + q[0]), my = 0.5 * (p[1] + q[1]);
        const double len = std::hypot(q[0] - p[0], q[1] - p[1]);
        double nx = (q[1] - p[1]) / len, ny = -(q[0] - p[0]) / len;
        if (nx * (mx - cx[L]) + ny * (my - cy[L]) < 0) {   // owner -> neighbour
            nx = -nx;
            ny = -ny;
        }
        for (int side = 0; side < (R >= 0 ? 2 : 1); ++side) {
            const int64_t c = side == 0 ? L : R;
            const int32_t other = side == 0 ? R : L;
            if (count[c] >= 3) {
                std::snprintf(err, errlen, "cell %lld has more than three faces", (long long)c);
                return false;
            }
            const int k = count[c]++;
            const double sg = side == 0 ? 1.0 : -1.0;
            g.nb[(size_t)k * nc + c] = other;
            G(TG_NX + k, c) = sg * nx;
            G(TG_NY + k, c) = sg * ny;
            G(TG_LW + k, c) = len / area[c];
            if (k < 2) {
                G(TG_AX + k, c) = mx - cx[c];
                G(TG_AY + k, c) = my - cy[c];
            }
            am[((size_t)k * 2 + 0) * nc + c] = mx - cx[c];
            am[((size_t)k * 2 + 1) * nc + c] = my - cy[c];
            G(TG_BX + k, c) = other >= 0 ? mx - cx[other] : 0.0;
            G(TG_BY + k, c) = other >= 0 ? my - cy[other] : 0.0;
            perim[c] += len;
        }
    }
    double rmin = 1e300;
    for (int64_t c = 0; c < nc; ++c) {
        if (count[c] != 3) {
            std::snprintf(err, errlen, "cell %lld has %d faces (a triangle has 3)", (long long)c, count[c]);
            return false;
        }
        rmin = std::min(rmin, 2.0 * area[c] / perim[c]);
        // gradient weights: grad U_c = sum_k W_k (U_k - U_c)
        double d[3][2], W[3][2];
        for (int k = 0; k < 3; ++k) {
            const double nx = G(TG_NX + k, c), ny = G(TG_NY + k, c);
            const double ax = am[((size_t)k * 2 + 0) * nc + c], ay = am[((size_t)k * 2 + 1) * nc + c];
            if (g.nb[(size_t)k * nc + c] >= 0) {   // the neighbour's centroid: (x_s - x_c) - (x_s - x_nb)
                d[k][0] = ax - G(TG_BX + k, c);
                d[k][1] = ay - G(TG_BY + k, c);
            } else {                                // the centroid's mirror image across the face
                const double hn = ax * nx + ay * ny;
                d[k][0] = 2.0 * hn * nx;
                d[k][1] = 2.0 * hn * ny;
            }
            W[k][0] = 0.5 * G(TG_LW + k, c) * nx;   // Green-Gauss
            W[k][1] = 0.5 * G(TG_LW + k, c) * ny;
        }
        if (gradient == GKS_GRAD_LSQ) {
            double M00 = 0, M01 = 0, M11 = 0;
            for (int k = 0; k < 3; ++k) {
                M00 += d[k][0] * d[k][0];
                M01 += d[k][0] * d[k][1];
                M11 += d[k][1] * d[k][1];
            }
            const double det = M00 * M11 - M01 * M01;
            if (!(det > 1e-14 * (M00 * M11))) {
                std::snprintf(err, errlen, "cell %lld: least-squares gradient fit is singular", (long long)c);
                return false;
            }
            for (int k = 0; k < 3; ++k) {
                W[k][0] = (M11 * d[k][0] - M01 * d[k][1]) / det;
                W[k][1] = (M00 * d[k][1] - M01 * d[k][0]) / det;
            }
        }
        for (int k = 0; k < 3; ++k) {
            G(TG_WX + k, c) = W[k][0];
            G(TG_WY + k, c) = W[k][1];
        }
    }
    g.area = std::move(area);
    g.rmin = rmin;
    return true;
}

}  // namespace gks
