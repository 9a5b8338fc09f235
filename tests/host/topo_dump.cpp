// Host-side check of the partition / N_x classification of libbidomain:
// builds bdm::Topology for a mesh given on the command line and prints the
// objects and per-subdomain dof counts in a line format the tests parse.
//   topo_dump nx ny nz px py pz cuts_x... cuts_y... cuts_z... [primal_space]
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2101_02959_amd/csrc/topology.hpp"

int main(int argc, char** argv) {
    if (argc < 7) return 2;
    int a = 1;
    const int nx = atoi(argv[a++]), ny = atoi(argv[a++]), nz = atoi(argv[a++]);
    const int px = atoi(argv[a++]), py = atoi(argv[a++]), pz = atoi(argv[a++]);
    const int nargs = 7 + (px + 1) + (py + 1) + (pz + 1);
    if (argc != nargs && argc != nargs + 1) return 2;
    std::vector<int> cx, cy, cz;
    for (int i = 0; i <= px; ++i) cx.push_back(atoi(argv[a++]));
    for (int i = 0; i <= py; ++i) cy.push_back(atoi(argv[a++]));
    for (int i = 0; i <= pz; ++i) cz.push_back(atoi(argv[a++]));
    bdm::Topology t;
    const int primal = argc == nargs + 1 ? atoi(argv[nargs]) : 0;
    const std::string err = t.build(nx, ny, nz, 0.01, px, py, pz, cx.data(), cy.data(), cz.data(), primal);
    if (!err.empty()) {
        printf("ERROR %s\n", err.c_str());
        return 1;
    }
    printf("COUNTS %zu %zu %zu %d\n", t.faces.size(), t.edges.size(), t.verts.size(), t.nprimal);
    const char* kinds[] = {"F", "E", "V"};
    for (const auto* v : {&t.faces, &t.edges, &t.verts})
        for (const auto& o : *v) {
            printf("OBJ %s", kinds[o.kind]);
            for (int s : o.subs) printf(" %d", s);
            printf(" |");
            for (int n : o.nodes) printf(" %d", n);
            printf("\n");
        }
    for (size_t s = 0; s < t.subs.size(); ++s) {
        const auto& b = t.subs[s];
        printf("SUB %zu %d %d %d %d %d %d |", s, b.nI, b.nr, b.nV, b.nc, b.nP, b.nIc);
        for (int n : b.I_nodes) printf(" %d", n);
        printf(" |");
        for (int n : b.r_nodes) printf(" %d", n);
        printf(" |");
        for (int p : b.primal) printf(" %d", p);
        printf("\n");
    }
    return 0;
}
