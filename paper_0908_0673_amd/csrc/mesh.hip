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
//
// First-order elements (Section 2.2: flat 3-node triangles, unknowns
// interpolated linearly between the corners) are carried as 6-node elements
// whose mid-side nodes are the edge midpoints, appended after the given
// nodes (three per element).  The quadratic map through them is the flat
// map, so geometry, tree and quadrature run unchanged; only the corners carry
// DOFs, the unknowns use the linear shape functions 1 - s - t, s, t (rule
// tables and correction integrals), and an element's mid-side slots refer to
// the DOFs of its corners 0, 1, 2 with shape function zero.
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
    const int na = m.linear ? 3 : 6;  // slots that carry DOFs
    const int32_t *el = m.h_elem.data();
    for (int64_t i = 0; i < 6 * ne; i++)
        BEM_REQUIRE(el[i] >= 0 && el[i] < nn, BEM_EINVAL, "element node index out of range");
    // node -> incidences (6 e + a, a < na), in element order
    std::vector<int64_t> start(nn + 1, 0);
    for (int64_t i = 0; i < 6 * ne; i++)
        if (i % 6 < na) start[el[i] + 1]++;
    for (int64_t g = 0; g < nn; g++) start[g + 1] += start[g];
    std::vector<int64_t> inc(start[nn]), fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < 6 * ne; i++)
        if (i % 6 < na) inc[fill[el[i]]++] = i;

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
        for (int a = 0; a < na; a++) {
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
    if (m.linear)  // mid-side slots: a corner's DOF, weighted by a zero shape function
        for (int64_t e = 0; e < ne; e++)
            for (int a = 3; a < 6; a++) m.h_elem_dofs[6 * e + a] = m.h_elem_dofs[6 * e + a - 3];
}

void load_mesh_host(bem_mesh &m, const double *xyz, int64_t n_nodes, const int32_t *elem, int64_t n_el, int nn,
                    double tol_deg) {
    BEM_REQUIRE(nn == 3 || nn == 6, BEM_EINVAL, "elements need 3 or 6 nodes");
    for (int64_t i = 0; i < (int64_t)nn * n_el; i++)
        BEM_REQUIRE(elem[i] >= 0 && elem[i] < n_nodes, BEM_EINVAL, "element node index out of range");
    m.n_el = n_el;
    m.linear = nn == 3;
    m.h_xyz.assign(xyz, xyz + 3 * n_nodes);
    for (double v : m.h_xyz) BEM_REQUIRE(std::isfinite(v), BEM_EINVAL, "non-finite node coordinate");
    if (nn == 6) {
        m.n_nodes = n_nodes;
        m.h_elem.assign(elem, elem + 6 * n_el);
    } else {
        m.n_nodes = n_nodes + 3 * n_el;
        m.h_xyz.resize(3 * m.n_nodes);
        m.h_elem.resize(6 * n_el);
        for (int64_t e = 0; e < n_el; e++)
            for (int j = 0; j < 3; j++) {
                const int64_t a = elem[3 * e + j], b = elem[3 * e + (j + 1) % 3], id = n_nodes + 3 * e + j;
                for (int d = 0; d < 3; d++) m.h_xyz[3 * id + d] = 0.5 * (xyz[3 * a + d] + xyz[3 * b + d]);
                m.h_elem[6 * e + j] = elem[3 * e + j];
                m.h_elem[6 * e + 3 + j] = (int32_t)id;  // mid-side of edge j, j + 1
            }
    }
    index_dofs(m, tol_deg);
}

}  // namespace bem
