// Host side of mesh loading: validation and sharp-edge DOF indexing
// (Section 2.3), then the upload of the mesh arrays.
//
// Indexing: elements are visited in order; at each node not yet indexed, the
// unit normals of every element holding the node (taken at the node, in
// element order) are grouped greedily: a normal joins the first group whose
// reference normal (the group's first member) lies within the tolerance angle,
// otherwise it starts a new group.  Each group is one DOF; its normal is the
// normalised sum of its members.  On a smooth surface every node gets one DOF;
// a cube edge node gets two and a corner three.
#include <cmath>

#include "kernels.h"

namespace bem {

namespace {

// Reference coordinates of the six nodes (corners, then mid-sides 01, 12, 20).
const double kNodeRef[6][2] = {{0, 0}, {1, 0}, {0, 1}, {0.5, 0}, {0.5, 0.5}, {0, 0.5}};

// Unit normal x_s x x_t / |x_s x x_t| of the quadratic map at (s, t); returns |x_s x x_t|.
double node_normal(const double *xyz, const int32_t *en, double s, double t, double n[3]) {
    double z = 1.0 - s - t;
    // d/ds and d/dt of the six quadratic shape functions
    double ds[6] = {-(4.0 * z - 1.0), 4.0 * s - 1.0, 0.0, 4.0 * (z - s), 4.0 * t, -4.0 * t};
    double dt[6] = {-(4.0 * z - 1.0), 0.0, 4.0 * t - 1.0, -4.0 * s, 4.0 * s, 4.0 * (z - t)};
    double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int k = 0; k < 6; k++) {
        const double *p = xyz + 3 * (int64_t)en[k];
        for (int d = 0; d < 3; d++) {
            a[d] += ds[k] * p[d];
            b[d] += dt[k] * p[d];
        }
    }
    double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double len = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    for (int d = 0; d < 3; d++) n[d] = len > 0 ? c[d] / len : 0.0;
    return len;
}

}  // namespace

void index_dofs(bem_mesh &m, double tol_deg) {
    const int64_t nn = m.n_nodes, ne = m.n_el;
    const int32_t *el = m.h_elem.data();
    for (int64_t i = 0; i < 6 * ne; i++)
        BEM_REQUIRE(el[i] >= 0 && el[i] < nn, BEM_EINVAL, "element node index out of range");
    // node -> incidences (6 e + a), in element order
    std::vector<int64_t> start(nn + 1, 0);
    for (int64_t i = 0; i < 6 * ne; i++) start[el[i] + 1]++;
    for (int64_t g = 0; g < nn; g++) start[g + 1] += start[g];
    std::vector<int64_t> inc(6 * ne), fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < 6 * ne; i++) inc[fill[el[i]]++] = i;

    // normals of every incidence
    std::vector<double> nrm(18 * ne);
    for (int64_t e = 0; e < ne; e++)
        for (int a = 0; a < 6; a++) {
            double J = node_normal(m.h_xyz.data(), el + 6 * e, kNodeRef[a][0], kNodeRef[a][1], &nrm[3 * (6 * e + a)]);
            BEM_REQUIRE(J > 0.0, BEM_EINVAL, "degenerate element " + std::to_string(e));
        }

    const double cos_tol = std::cos(tol_deg * M_PI / 180.0);
    m.h_elem_dofs.assign(6 * ne, -1);
    m.h_dof_node.clear();
    m.h_dof_normal.clear();
    std::vector<int64_t> group_ref;  // incidence holding each group's reference normal
    for (int64_t e = 0; e < ne; e++) {
        for (int a = 0; a < 6; a++) {
            if (m.h_elem_dofs[6 * e + a] >= 0) continue;
            const int32_t g = el[6 * e + a];
            const int64_t first = (int64_t)m.h_dof_node.size();
            for (int64_t p = start[g]; p < start[g + 1]; p++) {
                const int64_t ic = inc[p];
                const double *n = &nrm[3 * ic];
                int64_t grp = -1;
                for (int64_t q = first; q < (int64_t)m.h_dof_node.size(); q++) {
                    const double *r = &nrm[3 * group_ref[q]];
                    if (n[0] * r[0] + n[1] * r[1] + n[2] * r[2] > cos_tol) { grp = q; break; }
                }
                if (grp < 0) {
                    grp = (int64_t)m.h_dof_node.size();
                    m.h_dof_node.push_back(g);
                    group_ref.push_back(ic);
                    m.h_dof_normal.insert(m.h_dof_normal.end(), {0.0, 0.0, 0.0});
                }
                m.h_elem_dofs[ic] = (int32_t)grp;
                for (int d = 0; d < 3; d++) m.h_dof_normal[3 * grp + d] += n[d];
            }
        }
    }
    m.n_dof = (int64_t)m.h_dof_node.size();
    for (int64_t i = 0; i < m.n_dof; i++) {
        double *v = &m.h_dof_normal[3 * i];
        double l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int d = 0; d < 3; d++) v[d] /= l;
    }
}

}  // namespace bem
