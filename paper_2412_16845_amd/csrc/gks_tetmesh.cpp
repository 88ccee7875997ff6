// Tetrahedral-mesh ingest: topology checks and the geometry the tetrahedral kernels read.
//
// On 3D meshes each face is evaluated once, from its owner (face_cells[2s]): the D3Q4 lattice
// is chiral, so the flux of a face seen from the other side is not the negative of the owner's
// (Sec. 2.2 lattice, Sec. 3.1 rotation).  The face kernel stores the owner's flux, and each
// cell adds the fluxes of its four faces with the sign of its side.  Layouts (gks_internal.h):
//   per cell  nb[k]    neighbour across face slot k, or -(1 + bc) on a boundary face
//             W[k]     Green-Gauss gradient weight n_k |l_k| / (2 |Omega|) (outward normal)
//             N[k]     outward unit normal of slot k (for the PEC ghost of the gradient)
//             cf[k]    face id + 1 of slot k, negative when the cell is the face's neighbour
//             1/|Omega|
//   per face  n        unit normal owner -> neighbour
//             a, b     n3^2 / (1 + n1), n2 n3 / (1 + n1): with n they give the printed rotation T'
//                      (both 0 when n1 = -1, where T' = diag(-1, -1, 1))
//             |l|      area
//             x_s - x_L, x_s - x_R   (face centroid minus the cells' centroids; 0 on boundaries)
// Everything is computed in double precision (Sec. 3.1).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "gks_internal.h"

namespace gks {

bool build_tet_geometry(const gks_mesh_desc *m, TetGeometry &g, char *err, size_t errlen)
{
    const int64_t nv = m->nverts, nc = m->ncells, nf = m->nfaces;
    if (nv < 4 || nc < 1 || nf < 4) {
        std::snprintf(err, errlen, "a tetrahedral mesh needs >= 4 vertices, >= 1 cell and >= 4 faces");
        return false;
    }
    if (nc > (int64_t)0x1FFFFFFF || nf > (int64_t)0x3FFFFFFF || nv > (int64_t)0x7FFFFFFF) {
        std::snprintf(err, errlen, "mesh too large for 32-bit indexing");
        return false;
    }
    if (!m->vert_xy || !m->cell_verts || !m->face_cells || !m->face_verts) {
        std::snprintf(err, errlen, "vert_xy, cell_verts, face_cells and face_verts are required");
        return false;
    }
    const double *X = m->vert_xy;   // [3 * nverts] for tetrahedral meshes
    for (int64_t v = 0; v < 3 * nv; ++v)
        if (!std::isfinite(X[v])) {
            std::snprintf(err, errlen, "vertex %lld is not finite", (long long)(v / 3));
            return false;
        }
    std::vector<double> cen((size_t)3 * nc), vol(nc);
    for (int64_t c = 0; c < nc; ++c) {
        const int32_t *t = m->cell_verts + 4 * c;
        for (int k = 0; k < 4; ++k)
            if (t[k] < 0 || t[k] >= nv) {
                std::snprintf(err, errlen, "cell %lld has vertex %d outside [0, %lld)", (long long)c, t[k], (long long)nv);
                return false;
            }
        const double *p0 = X + 3 * t[0], *p1 = X + 3 * t[1], *p2 = X + 3 * t[2], *p3 = X + 3 * t[3];
        double a[3], b[3], d[3];
        for (int k = 0; k < 3; ++k) {
            a[k] = p1[k] - p0[k];
            b[k] = p2[k] - p0[k];
            d[k] = p3[k] - p0[k];
        }
        const double det = a[0] * (b[1] * d[2] - b[2] * d[1]) - a[1] * (b[0] * d[2] - b[2] * d[0]) +
                           a[2] * (b[0] * d[1] - b[1] * d[0]);
        vol[c] = std::fabs(det) / 6.0;
        if (!(vol[c] > 0)) {
            std::snprintf(err, errlen, "cell %lld is degenerate", (long long)c);
            return false;
        }
        for (int k = 0; k < 3; ++k) cen[3 * c + k] = 0.25 * (p0[k] + p1[k] + p2[k] + p3[k]);
    }
    auto has_vertex = [&](int64_t c, int32_t v) {
        const int32_t *t = m->cell_verts + 4 * c;
        return t[0] == v || t[1] == v || t[2] == v || t[3] == v;
    };
    std::vector<int32_t> count(nc, 0);
    std::vector<double> surf(nc, 0.0);
    g.ncell = nc;
    g.nface = nf;
    g.nb.assign((size_t)4 * nc, 0);
    g.cf.assign((size_t)4 * nc, 0);
    g.fc.assign((size_t)2 * nf, 0);
    g.cgeo.assign((size_t)TET_CGEO_ROWS * nc, 0.0);
    g.fgeo.assign((size_t)TET_FGEO_ROWS * nf, 0.0);
    auto C = [&](int row, int64_t c) -> double & { return g.cgeo[(size_t)row * nc + c]; };
    auto F = [&](int row, int64_t s) -> double & { return g.fgeo[(size_t)row * nf + s]; };
    for (int64_t s = 0; s < nf; ++s) {
        const int32_t L = m->face_cells[2 * s], R = m->face_cells[2 * s + 1];
        const int32_t *fv = m->face_verts + 3 * s;
        if (L < 0 || L >= nc) {
            std::snprintf(err, errlen, "face %lld: owner %d outside [0, %lld)", (long long)s, L, (long long)nc);
            return false;
        }
        if (R >= nc || R == L || (R < 0 && R != -(1 + GKS_BC_NONREFLECT) && R != -(1 + GKS_BC_PEC))) {
            std::snprintf(err, errlen, "face %lld: neighbour %d is neither a cell other than the owner nor a "
                                       "non-reflecting (-2) or PEC (-3) boundary", (long long)s, R);
            return false;
        }
        bool ok = fv[0] != fv[1] && fv[1] != fv[2] && fv[0] != fv[2];
        for (int k = 0; k < 3 && ok; ++k)
            ok = fv[k] >= 0 && fv[k] < nv && has_vertex(L, fv[k]) && (R < 0 || has_vertex(R, fv[k]));
        if (!ok) {
            std::snprintf(err, errlen, "face %lld: its vertices are not a face of its cells", (long long)s);
            return false;
        }
        const double *p = X + 3 * fv[0], *q = X + 3 * fv[1], *r = X + 3 * fv[2];
        double u[3], w[3], n[3], mid[3];
        for (int k = 0; k < 3; ++k) {
            u[k] = q[k] - p[k];
            w[k] = r[k] - p[k];
            mid[k] = (p[k] + q[k] + r[k]) / 3.0;
        }
        n[0] = u[1] * w[2] - u[2] * w[1];
        n[1] = u[2] * w[0] - u[0] * w[2];
        n[2] = u[0] * w[1] - u[1] * w[0];
        const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        const double area = 0.5 * nn;
        for (int k = 0; k < 3; ++k) n[k] /= nn;
        if (n[0] * (mid[0] - cen[3 * L]) + n[1] * (mid[1] - cen[3 * L + 1]) + n[2] * (mid[2] - cen[3 * L + 2]) < 0)
            for (int k = 0; k < 3; ++k) n[k] = -n[k];   // owner -> neighbour
        g.fc[2 * s] = L;
        g.fc[2 * s + 1] = R;
        for (int k = 0; k < 3; ++k) F(TF_N + k, s) = n[k];
        const double qd = 1.0 + n[0];
        F(TF_A, s) = (n[0] == -1.0) ? 0.0 : n[2] * n[2] / qd;
        F(TF_B, s) = (n[0] == -1.0) ? 0.0 : n[1] * n[2] / qd;
        F(TF_AREA, s) = area;
        for (int k = 0; k < 3; ++k) {
            F(TF_DL + k, s) = mid[k] - cen[3 * L + k];
            F(TF_DR + k, s) = R >= 0 ? mid[k] - cen[3 * R + k] : 0.0;
        }
        for (int side = 0; side < (R >= 0 ? 2 : 1); ++side) {
            const int64_t c = side == 0 ? L : R;
            const int32_t other = side == 0 ? R : L;
            if (count[c] >= 4) {
                std::snprintf(err, errlen, "cell %lld has more than four faces", (long long)c);
                return false;
            }
            const int k = count[c]++;
            const double sg = side == 0 ? 1.0 : -1.0;
            g.nb[(size_t)k * nc + c] = other;
            g.cf[(size_t)k * nc + c] = side == 0 ? (int32_t)(s + 1) : -(int32_t)(s + 1);
            for (int d = 0; d < 3; ++d) {
                C(TC_W + 3 * k + d, c) = 0.5 * sg * n[d] * area / vol[c];
                C(TC_N + 3 * k + d, c) = sg * n[d];
            }
            surf[c] += area;
        }
    }
    double rmin = 1e300;
    for (int64_t c = 0; c < nc; ++c) {
        if (count[c] != 4) {
            std::snprintf(err, errlen, "cell %lld has %d faces (a tetrahedron has 4)", (long long)c, count[c]);
            return false;
        }
        C(TC_IVOL, c) = 1.0 / vol[c];
        rmin = std::min(rmin, 3.0 * vol[c] / surf[c]);
    }
    g.vol = std::move(vol);
    g.rmin = rmin;
    return true;
}

}  // namespace gks
