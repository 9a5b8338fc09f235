// Host-side description of the structured slab and its box partition
// (Sec. 4.1 of the paper): subdomains, N_x equivalence classes (faces,
// edges, vertices), local dof orderings and the primal numbering.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace bdm {

struct Object {
    int kind;                   // 0 face, 1 edge, 2 vertex
    std::vector<int> subs;      // sharing subdomains, ascending
    std::vector<int> nodes;     // global node ids, ascending
};

struct SubInfo {
    int a, b, c;                // position in the subdomain grid
    int ex0, ex1, ey0, ey1, ez0, ez1;   // element box [e0, e1)
    // interior nodes (|N_x| = 1): first the core (interior nodes none of whose
    // 26 neighbours lies on the interface), then the rest; each part
    // ascending
    std::vector<int> I_nodes;
    std::vector<int> r_nodes;   // face nodes then edge nodes, object by object
    std::vector<int> V_nodes;   // vertex nodes
    std::vector<int> faces, edges, verts;     // object ids, ascending
    std::vector<int> face_off, edge_off;      // dof offset of each object in r
    // constraint index of each local face / edge (rows 2c, 2c+1 of C: the
    // averages of v and u_e over the object), -1 when the primal space does
    // not constrain it; edges come before faces
    std::vector<int> face_con, edge_con;
    int nI = 0, nr = 0, nV = 0, nG = 0, nc = 0, nP = 0;   // dof counts
    int nIc = 0;                // core dofs: the first nIc of the nI interior dofs
    std::vector<int> primal;    // local primal -> global primal
    // box-local node (i + (Lx+1)(j + (Ly+1)k)) -> local node index in [I|r|V]
    std::vector<int> lmap;
    int n() const { return nI + nG; }
    int Lx() const { return ex1 - ex0; }
    int Ly() const { return ey1 - ey0; }
    int Lz() const { return ez1 - ez0; }
};

struct Topology {
    int nx = 0, ny = 0, nz = 0;
    double h = 0;
    int px = 0, py = 0, pz = 0;
    std::vector<int> cx, cy, cz;
    int64_t N = 0;
    std::vector<Object> faces, edges, verts;
    std::vector<SubInfo> subs;
    // Primal space (Sec. 4.4): vertex values always; the averages over every
    // edge and over every face when cons_edges / cons_faces.  Global primal
    // numbering: (v, u_e) per vertex, then the two averages per constrained
    // edge, then per constrained face.
    bool cons_edges = true, cons_faces = false;
    int nprimal = 0;
    std::vector<int> pobj_node;   // first node of each primal object, in numbering order

    // primal_space: 0 vertices + edges, 1 vertices, 2 vertices + edges + faces.
    // Returns an empty string on success, else a message.
    std::string build(int nx, int ny, int nz, double h, int px, int py, int pz,
                      const int* cuts_x, const int* cuts_y, const int* cuts_z, int primal_space = 0);
    int64_t node(int i, int j, int k) const {
        return i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k);
    }
    int sid(int a, int b, int c) const { return a + px * (b + py * c); }
};

}  // namespace bdm
