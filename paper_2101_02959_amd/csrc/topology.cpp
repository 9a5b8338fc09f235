// Partition and N_x classification for a tensor-product box partition.
//
// Interface objects follow directly from the cut planes: a node lying on
// exactly one interior cut plane belongs to a face (2 subdomains), on two to
// an edge (4 subdomains), on three to a vertex (8 subdomains).  Nodes on the
// physical (Neumann) boundary that lie on no interior cut are interior to
// their subdomain (Sec. 4.1).  Objects of each kind are ordered by their
// smallest node id.
#include "topology.hpp"

#include <algorithm>
#include <numeric>

namespace bdm {

namespace {

// Coordinates of part p along an axis that lie on no interior cut.
inline void open_range(const std::vector<int>& c, int p, int& lo, int& hi) {
    const int P = (int)c.size() - 1;
    lo = c[p] + (p > 0 ? 1 : 0);
    hi = c[p + 1] - (p + 1 < P ? 1 : 0);
}

std::vector<char> cut_mask(const std::vector<int>& c, int n) {
    std::vector<char> m(n + 1, 0);
    for (size_t a = 1; a + 1 < c.size(); ++a) m[c[a]] = 1;
    return m;
}

void sort_objects(std::vector<Object>& v) {
    std::sort(v.begin(), v.end(),
              [](const Object& x, const Object& y) { return x.nodes[0] < y.nodes[0]; });
}

}  // namespace

std::string Topology::build(int nx_, int ny_, int nz_, double h_, int px_, int py_, int pz_,
                            const int* cuts_x, const int* cuts_y, const int* cuts_z, int primal_space) {
    nx = nx_; ny = ny_; nz = nz_; h = h_; px = px_; py = py_; pz = pz_;
    if (primal_space < 0 || primal_space > 2) return "unknown primal space";
    cons_edges = primal_space != 1;
    cons_faces = primal_space == 2;
    if (nx < 2 || ny < 2 || nz < 2 || !(h > 0)) return "mesh sizes must be >= 2 and h > 0";
    if (px < 2 || py < 2 || pz < 2) return "need >= 2 subdomains per axis";
    cx.assign(cuts_x, cuts_x + px + 1);
    cy.assign(cuts_y, cuts_y + py + 1);
    cz.assign(cuts_z, cuts_z + pz + 1);
    auto check = [](const std::vector<int>& c, int n) {
        if (c.front() != 0 || c.back() != n) return false;
        for (size_t a = 1; a < c.size(); ++a)
            if (c[a] <= c[a - 1]) return false;
        return true;
    };
    if (!check(cx, nx) || !check(cy, ny) || !check(cz, nz))
        return "cuts must increase strictly from 0 to n";
    N = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    if (N > (int64_t)INT32_MAX / 2) return "mesh too large";

    faces.clear(); edges.clear(); verts.clear();
    int lo, hi, lo2, hi2;
    // faces normal to x, y, z
    for (int a = 1; a < px; ++a)
        for (int b = 0; b < py; ++b)
            for (int c = 0; c < pz; ++c) {
                Object o{0, {sid(a - 1, b, c), sid(a, b, c)}, {}};
                open_range(cy, b, lo, hi);
                open_range(cz, c, lo2, hi2);
                for (int k = lo2; k <= hi2; ++k)
                    for (int j = lo; j <= hi; ++j) o.nodes.push_back((int)node(cx[a], j, k));
                faces.push_back(std::move(o));
            }
    for (int a = 0; a < px; ++a)
        for (int b = 1; b < py; ++b)
            for (int c = 0; c < pz; ++c) {
                Object o{0, {sid(a, b - 1, c), sid(a, b, c)}, {}};
                open_range(cx, a, lo, hi);
                open_range(cz, c, lo2, hi2);
                for (int k = lo2; k <= hi2; ++k)
                    for (int i = lo; i <= hi; ++i) o.nodes.push_back((int)node(i, cy[b], k));
                faces.push_back(std::move(o));
            }
    for (int a = 0; a < px; ++a)
        for (int b = 0; b < py; ++b)
            for (int c = 1; c < pz; ++c) {
                Object o{0, {sid(a, b, c - 1), sid(a, b, c)}, {}};
                open_range(cx, a, lo, hi);
                open_range(cy, b, lo2, hi2);
                for (int j = lo2; j <= hi2; ++j)
                    for (int i = lo; i <= hi; ++i) o.nodes.push_back((int)node(i, j, cz[c]));
                faces.push_back(std::move(o));
            }
    // edges along x, y, z
    for (int a = 0; a < px; ++a)
        for (int b = 1; b < py; ++b)
            for (int c = 1; c < pz; ++c) {
                Object o{1, {sid(a, b - 1, c - 1), sid(a, b, c - 1), sid(a, b - 1, c), sid(a, b, c)}, {}};
                open_range(cx, a, lo, hi);
                for (int i = lo; i <= hi; ++i) o.nodes.push_back((int)node(i, cy[b], cz[c]));
                edges.push_back(std::move(o));
            }
    for (int a = 1; a < px; ++a)
        for (int b = 0; b < py; ++b)
            for (int c = 1; c < pz; ++c) {
                Object o{1, {sid(a - 1, b, c - 1), sid(a, b, c - 1), sid(a - 1, b, c), sid(a, b, c)}, {}};
                open_range(cy, b, lo, hi);
                for (int j = lo; j <= hi; ++j) o.nodes.push_back((int)node(cx[a], j, cz[c]));
                edges.push_back(std::move(o));
            }
    for (int a = 1; a < px; ++a)
        for (int b = 1; b < py; ++b)
            for (int c = 0; c < pz; ++c) {
                Object o{1, {sid(a - 1, b - 1, c), sid(a, b - 1, c), sid(a - 1, b, c), sid(a, b, c)}, {}};
                open_range(cz, c, lo, hi);
                for (int k = lo; k <= hi; ++k) o.nodes.push_back((int)node(cx[a], cy[b], k));
                edges.push_back(std::move(o));
            }
    for (int c = 1; c < pz; ++c)
        for (int b = 1; b < py; ++b)
            for (int a = 1; a < px; ++a) {
                Object o{2, {}, {(int)node(cx[a], cy[b], cz[c])}};
                for (int dc = -1; dc <= 0; ++dc)
                    for (int db = -1; db <= 0; ++db)
                        for (int da = -1; da <= 0; ++da) o.subs.push_back(sid(a + da, b + db, c + dc));
                verts.push_back(std::move(o));
            }
    for (auto* v : {&faces, &edges, &verts})
        for (auto& o : *v) std::sort(o.subs.begin(), o.subs.end());
    sort_objects(faces);
    sort_objects(edges);
    sort_objects(verts);
    const int edge_p0 = 2 * (int)verts.size();
    const int face_p0 = edge_p0 + (cons_edges ? 2 * (int)edges.size() : 0);
    nprimal = face_p0 + (cons_faces ? 2 * (int)faces.size() : 0);
    pobj_node.clear();
    for (auto& o : verts) pobj_node.push_back(o.nodes[0]);
    if (cons_edges)
        for (auto& o : edges) pobj_node.push_back(o.nodes[0]);
    if (cons_faces)
        for (auto& o : faces) pobj_node.push_back(o.nodes[0]);

    const int nsub = px * py * pz;
    subs.assign(nsub, SubInfo());
    for (int c = 0; c < pz; ++c)
        for (int b = 0; b < py; ++b)
            for (int a = 0; a < px; ++a) {
                SubInfo& s = subs[sid(a, b, c)];
                s.a = a; s.b = b; s.c = c;
                s.ex0 = cx[a]; s.ex1 = cx[a + 1];
                s.ey0 = cy[b]; s.ey1 = cy[b + 1];
                s.ez0 = cz[c]; s.ez1 = cz[c + 1];
            }
    for (int f = 0; f < (int)faces.size(); ++f)
        for (int s : faces[f].subs) subs[s].faces.push_back(f);
    for (int e = 0; e < (int)edges.size(); ++e)
        for (int s : edges[e].subs) subs[s].edges.push_back(e);
    for (int v = 0; v < (int)verts.size(); ++v)
        for (int s : verts[v].subs) subs[s].verts.push_back(v);

    const std::vector<char> mx = cut_mask(cx, nx), my = cut_mask(cy, ny), mz = cut_mask(cz, nz);
    for (int sidx = 0; sidx < nsub; ++sidx) {
        SubInfo& s = subs[sidx];
        // An interior node couples (through the elements around it) with its 26
        // neighbours only, all inside the box; a core node has none of them on
        // a cut plane, so its rows of K_IG are zero.
        s.I_nodes.clear();
        std::vector<int> shell;
        for (int k = s.ez0; k <= s.ez1; ++k)
            for (int j = s.ey0; j <= s.ey1; ++j)
                for (int i = s.ex0; i <= s.ex1; ++i) {
                    if (mx[i] || my[j] || mz[k]) continue;
                    bool core = true;
                    for (int dz = -1; dz <= 1 && core; ++dz)
                        for (int dy = -1; dy <= 1 && core; ++dy)
                            for (int dx = -1; dx <= 1 && core; ++dx) {
                                const int ii = i + dx, jj = j + dy, kk = k + dz;
                                if (ii < 0 || ii > nx || jj < 0 || jj > ny || kk < 0 || kk > nz) continue;
                                if (mx[ii] || my[jj] || mz[kk]) core = false;
                            }
                    (core ? s.I_nodes : shell).push_back((int)node(i, j, k));
                }
        s.nIc = 2 * (int)s.I_nodes.size();
        s.I_nodes.insert(s.I_nodes.end(), shell.begin(), shell.end());
        s.r_nodes.clear();
        s.face_off.clear();
        s.edge_off.clear();
        for (int f : s.faces) {
            s.face_off.push_back(2 * (int)s.r_nodes.size());
            s.r_nodes.insert(s.r_nodes.end(), faces[f].nodes.begin(), faces[f].nodes.end());
        }
        for (int e : s.edges) {
            s.edge_off.push_back(2 * (int)s.r_nodes.size());
            s.r_nodes.insert(s.r_nodes.end(), edges[e].nodes.begin(), edges[e].nodes.end());
        }
        s.V_nodes.clear();
        for (int v : s.verts) s.V_nodes.push_back(verts[v].nodes[0]);
        s.nI = 2 * (int)s.I_nodes.size();
        s.nr = 2 * (int)s.r_nodes.size();
        s.nV = 2 * (int)s.V_nodes.size();
        s.nG = s.nr + s.nV;
        s.primal.clear();
        for (int v : s.verts) { s.primal.push_back(2 * v); s.primal.push_back(2 * v + 1); }
        int ncon = 0;
        s.edge_con.assign(s.edges.size(), -1);
        s.face_con.assign(s.faces.size(), -1);
        if (cons_edges)
            for (size_t t = 0; t < s.edges.size(); ++t) {
                s.edge_con[t] = ncon++;
                s.primal.push_back(edge_p0 + 2 * s.edges[t]);
                s.primal.push_back(edge_p0 + 2 * s.edges[t] + 1);
            }
        if (cons_faces)
            for (size_t t = 0; t < s.faces.size(); ++t) {
                s.face_con[t] = ncon++;
                s.primal.push_back(face_p0 + 2 * s.faces[t]);
                s.primal.push_back(face_p0 + 2 * s.faces[t] + 1);
            }
        s.nc = 2 * ncon;
        s.nP = s.nV + s.nc;
        // box-local map
        const int Lx1 = s.Lx() + 1, Ly1 = s.Ly() + 1, Lz1 = s.Lz() + 1;
        s.lmap.assign((size_t)Lx1 * Ly1 * Lz1, -1);
        auto put = [&](int gnode, int lidx) {
            int i = (int)(gnode % (nx + 1));
            int j = (int)((gnode / (nx + 1)) % (ny + 1));
            int k = (int)(gnode / ((int64_t)(nx + 1) * (ny + 1)));
            s.lmap[(i - s.ex0) + Lx1 * ((j - s.ey0) + Ly1 * (k - s.ez0))] = lidx;
        };
        int q = 0;
        for (int g : s.I_nodes) put(g, q++);
        for (int g : s.r_nodes) put(g, q++);
        for (int g : s.V_nodes) put(g, q++);
        for (int x : s.lmap)
            if (x < 0) return "internal error: box node not classified";
    }
    return "";
}

}  // namespace bdm
