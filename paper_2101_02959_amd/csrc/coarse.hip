// FP64 coarse problem of BDDC / FETI-DP (paper Sec. 4.4): the assembled
// primal matrix S_PiPi over vertex values and the edge (and face) averages.
//
// The matrix couples two primal objects when they share a subdomain, so the
// cut planes of the subdomain grid are separators: the objects lying on the
// plane x = X (vertices, y- and z-edges, x-faces there) separate those of the
// subdomain columns left of X from those right of it.  Recursive bisection of
// the subdomain grid along its longest axis gives a nested-dissection order
// and its elimination tree of fronts; boxes of at most 64 subdomains are the
// leaves.  Each front holds its eliminated objects (the separator, or all
// objects inside a leaf box) followed by its boundary objects (those on the
// box faces that belong to its subdomains).
//
// Factorisation (multifrontal Cholesky, bottom up, all fronts of one height
// at once): leaf fronts receive the subdomain blocks S_PiPi^(j) (scattered
// colour by colour so that no two writers meet), inner fronts the update
// matrices of their two children (extend-add, one launch per child slot); the
// eliminated block is factored and the boundary block receives the Schur
// update by the batched panel / rank-k kernels of the local factorisations.
// The singular direction (u_e constant) is removed by pinning one u_e primal:
// its row and column are left out and its diagonal set to 1.
//
// Each front is stored with n_e extra rows below it that start as the
// identity in the eliminated columns: the same partial factorisation then
// leaves X = L_ee^{-T} in those rows (X = I L_ee^{-T}, exactly as it leaves
// L_be = F_be L_ee^{-T} in the boundary rows), so every triangular solve of
// the coarse solve becomes a wide matrix-vector product:
//   forward (bottom up)  y = L_ee^{-1} z_e = X^T z_e,  z_b -= L_be y,
//                        z_b then travels to the parent (extend-add);
//   backward (top down)  x_e = L_ee^{-T} (y - L_be^T x_b) = X t.
#include <algorithm>
#include <cstdlib>
#include <functional>
#include <vector>

#include "coarse.hpp"
#include "kernels.hpp"

namespace bdm {

namespace {

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Leaf assembly: F[pa, pb] += S^(s)[a, b] on the lower triangle of the leaf
// front of subdomain s (one colour per launch).
__global__ void k_nd_leaf_assemble(const int* __restrict__ list, const int* __restrict__ nPv,
                                   const double* __restrict__ Sp, int sp_stride, const int* __restrict__ sub_pos,
                                   int maxp, const int* __restrict__ sub_front, const int64_t* __restrict__ foff,
                                   const int* __restrict__ ldv, double* __restrict__ F) {
    const int s = list[blockIdx.x];
    const int nP = nPv[s];
    const int f = sub_front[s];
    double* Ff = F + foff[f];
    const int64_t ld = ldv[f];
    const int* pos = sub_pos + (int64_t)s * maxp;
    const double* S = Sp + (int64_t)s * sp_stride;
    for (int idx = threadIdx.x; idx < nP * nP; idx += blockDim.x) {
        const int a = idx % nP, b = idx / nP;
        const int pa = pos[a], pb = pos[b];
        if (pa < 0 || pb < 0 || pa < pb) continue;
        Ff[pa + pb * ld] += S[a + b * nP];
    }
}

// Extend-add of update matrices: child c's trailing block (lower triangle)
// into its parent, column j per workgroup row.
__global__ void k_nd_extend(const int* __restrict__ kids, const int* __restrict__ parent,
                            const int64_t* __restrict__ foff, const int* __restrict__ nev, const int* __restrict__ mv,
                            const int* __restrict__ ldv, const int64_t* __restrict__ pmoff,
                            const int* __restrict__ pmap, double* __restrict__ F) {
    const int c = kids[blockIdx.y];
    const int ne = nev[c], nbd = mv[c] - ne;
    const int j = blockIdx.x;
    if (j >= nbd) return;
    const int p = parent[c];
    const int64_t ldc = ldv[c], ldp = ldv[p];
    const int* map = pmap + pmoff[c];
    const double* Fc = F + foff[c];
    double* Fp = F + foff[p];
    const int Q = map[j];
    for (int i = j + threadIdx.x; i < nbd; i += blockDim.x) {
        const int P = map[i];
        const int r = max(P, Q), q = min(P, Q);
        Fp[r + q * ldp] += Fc[(ne + i) + (ne + j) * ldc];
    }
}

// identity in the extra rows: F[m + i, i] = 1, i < n_e
__global__ void k_nd_eye(const int64_t* __restrict__ foff, const int* __restrict__ nev, const int* __restrict__ mv,
                         const int* __restrict__ ldv, double* __restrict__ F) {
    const int f = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nev[f]) return;
    F[foff[f] + (mv[f] + i) + (int64_t)i * ldv[f]] = 1.0;
}

// Front blocks for the solve: blk 0 = X (rows [m, m + n_e)), blk 1 = L_be
// (rows [n_e, m)); both have the n_e eliminated columns.
__device__ inline void nd_block(int blk, int ne, int m, int& r0, int& R) {
    if (blk == 0) { r0 = m; R = ne; } else { r0 = ne; R = m - ne; }
}

// out[c] = base[c] + sgn * sum_r B[r][c] x[r], c < n_e (one wave per column);
// x is the front's eliminated part for blk 0 and its boundary part for blk 1.
__global__ __launch_bounds__(256) void k_nd_gemv_t(const int64_t* __restrict__ foff, const int* __restrict__ nev,
                                                   const int* __restrict__ mv, const int* __restrict__ ldv, int blk,
                                                   const double* __restrict__ F, const int64_t* __restrict__ zoff,
                                                   const double* __restrict__ xv, const double* __restrict__ base,
                                                   double* __restrict__ out, double sgn) {
    const int f = blockIdx.y;
    const int ne = nev[f], m = mv[f];
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (c >= ne) return;
    int r0, R;
    nd_block(blk, ne, m, r0, R);
    const int64_t ld = ldv[f];
    const double* col = F + foff[f] + r0 + c * ld;
    const double* x = xv + zoff[f] + (blk ? ne : 0);
    double acc = 0.0;
    for (int r = lane; r < R; r += 64) acc += col[r] * x[r];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
        const int64_t k = zoff[f] + c;
        out[k] = (base ? base[k] : 0.0) + sgn * acc;
    }
}

// out[r] = base[r] + sgn * sum_c B[r][c] x[c] over the n_e columns, GN_RB
// rows per workgroup and GN_CS column slices (a wave reads four columns of
// 16 rows, four columns in flight per thread), the slices summed in LDS in a
// fixed order; rows of blk 1 land at the front's boundary part.  Narrow row
// blocks keep enough workgroups in flight on the few large fronts near the
// root of the tree.
constexpr int GN_RB = 16, GN_CS = 256 / GN_RB;
__global__ __launch_bounds__(256) void k_nd_gemv_n(const int64_t* __restrict__ foff, const int* __restrict__ nev,
                                                   const int* __restrict__ mv, const int* __restrict__ ldv, int blk,
                                                   const double* __restrict__ F, const int64_t* __restrict__ zoff,
                                                   const double* __restrict__ xv, const double* __restrict__ base,
                                                   double* __restrict__ out, double sgn) {
    __shared__ double red[GN_CS][GN_RB + 1];
    const int f = blockIdx.y;
    const int ne = nev[f], m = mv[f];
    int r0, R;
    nd_block(blk, ne, m, r0, R);
    if ((int)blockIdx.x * GN_RB >= R) return;
    const int rl = threadIdx.x % GN_RB, cs = threadIdx.x / GN_RB;
    const int row = blockIdx.x * GN_RB + rl, rc = min(row, R - 1);
    const int64_t ld = ldv[f];
    const double* A = F + foff[f] + r0 + rc;
    const double* x = xv + zoff[f];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int c = cs;
    for (; c + 3 * GN_CS < ne; c += 4 * GN_CS) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += A[(int64_t)(c + u * GN_CS) * ld] * x[c + u * GN_CS];
    }
    for (; c < ne; c += GN_CS) acc[0] += A[(int64_t)c * ld] * x[c];
    red[cs][rl] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (threadIdx.x < GN_RB && row < R) {
        double d = 0.0;
#pragma unroll
        for (int q = 0; q < GN_CS; ++q) d += red[q][rl];
        const int64_t k = zoff[f] + (blk ? ne : 0) + row;
        out[k] = (base ? base[k] : 0.0) + sgn * d;
    }
}

__global__ void k_nd_set_one(double* __restrict__ F, int64_t idx) { F[idx] = 1.0; }

__global__ void k_nd_info(int n, const int* __restrict__ flags, int* __restrict__ out) {
    int bad = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) bad |= flags[i];
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0 && bad) out[0] = 1;
}

// z_f = (b at the eliminated dofs, 0 at the boundary dofs)
__global__ void k_nd_gather_e(const int64_t* __restrict__ zoff, const int* __restrict__ nev,
                              const int* __restrict__ mv, const int* __restrict__ vars, const double* __restrict__ b,
                              double* __restrict__ z) {
    const int f = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= mv[f]) return;
    const int64_t o = zoff[f] + t;
    z[o] = t < nev[f] ? b[vars[o]] : 0.0;
}

// z_f[boundary] = x at the boundary dofs (known from the fronts above)
__global__ void k_nd_gather_b(const int64_t* __restrict__ zoff, const int* __restrict__ nev,
                              const int* __restrict__ mv, const int* __restrict__ vars, const double* __restrict__ x,
                              double* __restrict__ z) {
    const int f = blockIdx.y;
    const int t = nev[f] + blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= mv[f]) return;
    const int64_t o = zoff[f] + t;
    z[o] = x[vars[o]];
}

__global__ void k_nd_scatter_e(const int64_t* __restrict__ zoff, const int* __restrict__ nev,
                               const int* __restrict__ vars, const double* __restrict__ z, double* __restrict__ x) {
    const int f = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nev[f]) return;
    const int64_t o = zoff[f] + t;
    x[vars[o]] = z[o];
}

// parent z += child update vector (child boundary part)
__global__ void k_nd_extend_vec(const int* __restrict__ kids, const int* __restrict__ parent,
                                const int64_t* __restrict__ zoff, const int* __restrict__ nev,
                                const int* __restrict__ mv, const int64_t* __restrict__ pmoff,
                                const int* __restrict__ pmap, double* __restrict__ z) {
    const int c = kids[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int ne = nev[c];
    if (i >= mv[c] - ne) return;
    z[zoff[parent[c]] + pmap[pmoff[c] + i]] += z[zoff[c] + ne + i];
}

}  // namespace

// ------------------------------------------------------------------ symbolic
std::string CoarseSolver::init(const Topology& t, int pin_, int maxp_) {
    np = t.nprimal;
    pin = pin_;
    maxp = maxp_;
    const int nobj = (int)t.pobj_node.size();
    if (2 * nobj != np) return "internal error: primal numbering is not two dofs per primal object";
    if (np == 0) return "no primal unknowns";
    // doubled subdomain-grid coordinates: cut plane a -> 2a, slab a -> 2a + 1
    auto dbl = [](int n, const std::vector<int>& cuts) {
        std::vector<int> c(n + 1, 0);
        int a = 0;
        for (int i = 0; i <= n; ++i) {
            while (a + 1 < (int)cuts.size() && cuts[a + 1] <= i) ++a;
            c[i] = (cuts[a] == i) ? 2 * a : 2 * a + 1;
        }
        return c;
    };
    const std::vector<int> dx = dbl(t.nx, t.cx), dy = dbl(t.ny, t.cy), dz = dbl(t.nz, t.cz);
    std::vector<int> oc(3 * (size_t)nobj);
    for (int o = 0; o < nobj; ++o) {
        const int node = t.pobj_node[o];
        const int i = node % (t.nx + 1), j = (node / (t.nx + 1)) % (t.ny + 1), k = node / ((t.nx + 1) * (t.ny + 1));
        oc[3 * o] = dx[i];
        oc[3 * o + 1] = dy[j];
        oc[3 * o + 2] = dz[k];
    }
    // objects of each subdomain
    const int nsub = (int)t.subs.size();
    std::vector<std::vector<int>> sobj(nsub);
    for (int q = 0; q < nsub; ++q) {
        for (int p : t.subs[q].primal) sobj[q].push_back(p / 2);
        std::sort(sobj[q].begin(), sobj[q].end());
        sobj[q].erase(std::unique(sobj[q].begin(), sobj[q].end()), sobj[q].end());
    }
    struct Tmp {
        std::vector<int> elim, bnd;
        int kid[2] = {-1, -1};
        int height = 0;
    };
    std::vector<Tmp> tf;
    std::vector<int> mark(nobj, -1), leaf_of(nsub, -1);
    // largest leaf box (subdomains): 4 x 4 x 4 leaves, measured against 2 x 2 x 2
    // (12 against 9 tree levels at 32 x 32 x 16 subdomains, whose per-level
    // launches dominate the upper levels); BDM_COARSE_LEAF_SUBS overrides
    int64_t leaf_max = 64;
    if (const char* e = std::getenv("BDM_COARSE_LEAF_SUBS")) leaf_max = std::max(1, std::atoi(e));
    int stampc = 0;
    std::function<int(const int*, const int*, std::vector<int>&)> nd =
        [&](const int* lo, const int* hi, std::vector<int>& inner) -> int {
        const int ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
        int ax = 0;
        for (int d = 1; d < 3; ++d)
            if (ext[d] > ext[ax]) ax = d;
        Tmp fr;
        if ((int64_t)ext[0] * ext[1] * ext[2] <= leaf_max || ext[ax] < 2) {
            fr.elim = inner;
            const int st = stampc++;
            for (int o : inner) mark[o] = st;
            const int id = (int)tf.size();
            for (int c = lo[2]; c < hi[2]; ++c)
                for (int b = lo[1]; b < hi[1]; ++b)
                    for (int a = lo[0]; a < hi[0]; ++a) {
                        const int q = t.sid(a, b, c);
                        leaf_of[q] = id;
                        for (int o : sobj[q])
                            if (mark[o] != st) {
                                mark[o] = st;
                                fr.bnd.push_back(o);
                            }
                    }
            std::sort(fr.bnd.begin(), fr.bnd.end());
            tf.push_back(std::move(fr));
            return id;
        }
        const int M = (lo[ax] + hi[ax]) / 2;
        std::vector<int> L, R;
        for (int o : inner) {
            const int x = oc[3 * o + ax];
            if (x == 2 * M) fr.elim.push_back(o);
            else if (x < 2 * M) L.push_back(o);
            else R.push_back(o);
        }
        std::vector<int>().swap(inner);
        int lo2[3] = {lo[0], lo[1], lo[2]}, hi1[3] = {hi[0], hi[1], hi[2]};
        hi1[ax] = M;
        lo2[ax] = M;
        const int cl = nd(lo, hi1, L);
        const int cr = nd(lo2, hi, R);
        const int st = stampc++;
        for (int o : fr.elim) mark[o] = st;
        for (int cidx : {cl, cr})
            for (int o : tf[cidx].bnd)
                if (mark[o] != st) {
                    mark[o] = st;
                    fr.bnd.push_back(o);
                }
        std::sort(fr.bnd.begin(), fr.bnd.end());
        fr.kid[0] = cl;
        fr.kid[1] = cr;
        fr.height = 1 + std::max(tf[cl].height, tf[cr].height);
        tf.push_back(std::move(fr));
        return (int)tf.size() - 1;
    };
    std::vector<int> all;
    for (int o = 0; o < nobj; ++o) all.push_back(o);
    const int lo[3] = {0, 0, 0}, hi[3] = {t.px, t.py, t.pz};
    const int root = nd(lo, hi, all);
    if (!tf[root].bnd.empty()) return "internal error: coarse root front has boundary objects";
    for (int q = 0; q < nsub; ++q)
        if (leaf_of[q] < 0) return "internal error: subdomain outside the coarse leaves";
    // renumber height by height
    nfront = (int)tf.size();
    H = 0;
    for (auto& f : tf) H = std::max(H, f.height + 1);
    hptr.assign(H + 1, 0);
    for (auto& f : tf) ++hptr[f.height + 1];
    for (int h = 0; h < H; ++h) hptr[h + 1] += hptr[h];
    std::vector<int> nid(nfront), fill(hptr.begin(), hptr.end() - 1);
    for (int f = 0; f < nfront; ++f) nid[f] = fill[tf[f].height]++;
    ne.assign(nfront, 0);
    m.assign(nfront, 0);
    ld.assign(nfront, 0);
    parent.assign(nfront, -1);
    foff.assign(nfront, 0);
    zoff.assign(nfront, 0);
    pmoff.assign(nfront, 0);
    std::vector<std::vector<int>> fv(nfront);
    for (int f = 0; f < nfront; ++f) {
        const int g = nid[f];
        for (int o : tf[f].elim) { fv[g].push_back(2 * o); fv[g].push_back(2 * o + 1); }
        ne[g] = (int)fv[g].size();
        for (int o : tf[f].bnd) { fv[g].push_back(2 * o); fv[g].push_back(2 * o + 1); }
        m[g] = (int)fv[g].size();
        ld[g] = m[g] + ne[g];
        for (int s = 0; s < 2; ++s)
            if (tf[f].kid[s] >= 0) parent[nid[tf[f].kid[s]]] = g;
    }
    kids[0].assign(H, {});
    kids[1].assign(H, {});
    for (int f = 0; f < nfront; ++f)
        for (int s = 0; s < 2; ++s)
            if (tf[f].kid[s] >= 0) kids[s][tf[f].height].push_back(nid[tf[f].kid[s]]);
    int64_t aF = 0, aZ = 0, aP = 0;
    for (int g = 0; g < nfront; ++g) {
        foff[g] = aF; aF += (int64_t)ld[g] * m[g];
        zoff[g] = aZ; aZ += m[g];
        pmoff[g] = aP; if (parent[g] >= 0) aP += m[g] - ne[g];
    }
    nF = std::max<int64_t>(aF, 1);
    nZ = std::max<int64_t>(aZ, 1);
    vars.assign(std::max<int64_t>(aZ, 1), 0);
    pmap.assign(std::max<int64_t>(aP, 1), 0);
    for (int g = 0; g < nfront; ++g)
        std::copy(fv[g].begin(), fv[g].end(), vars.begin() + zoff[g]);
    std::vector<int> posv(np, -1);
    for (int g = 0; g < nfront; ++g) {
        const int p = parent[g];
        if (p < 0) continue;
        for (int u = 0; u < m[p]; ++u) posv[fv[p][u]] = u;
        for (int i = ne[g]; i < m[g]; ++i) {
            const int u = posv[fv[g][i]];
            if (u < 0) return "internal error: coarse child variable missing from its parent";
            pmap[pmoff[g] + i - ne[g]] = u;
        }
        for (int u = 0; u < m[p]; ++u) posv[fv[p][u]] = -1;
    }
    // subdomain -> leaf front positions; the pin
    sub_front.assign(nsub, 0);
    sub_pos.assign((size_t)nsub * maxp, -1);
    for (int q = 0; q < nsub; ++q) {
        const int g = nid[leaf_of[q]];
        sub_front[q] = g;
        for (int u = 0; u < m[g]; ++u) posv[fv[g][u]] = u;
        const auto& pr = t.subs[q].primal;
        if ((int)pr.size() > maxp) return "internal error: too many primal dofs in a subdomain";
        for (size_t a = 0; a < pr.size(); ++a) {
            const int u = posv[pr[a]];
            if (u < 0) return "internal error: subdomain primal missing from its leaf front";
            sub_pos[(size_t)q * maxp + a] = (pr[a] == pin) ? -1 : u;
        }
        for (int u = 0; u < m[g]; ++u) posv[fv[g][u]] = -1;
    }
    for (int g = 0; g < nfront && pin_front < 0; ++g)
        for (int u = 0; u < ne[g]; ++u)
            if (fv[g][u] == pin) { pin_front = g; pin_pos = u; break; }
    if (pin_front < 0) return "internal error: pinned primal not eliminated";
    // launch sizes per height
    const int w = interior_panel_width();
    maxne.assign(H, 0); maxm.assign(H, 0); maxnb.assign(H, 0); schur_tiles.assign(H, 0);
    trail_tiles.assign(H, {}); panel_rows.assign(H, {});
    maxnf = 1;
    for (int h = 0; h < H; ++h) {
        maxnf = std::max(maxnf, hptr[h + 1] - hptr[h]);
        for (int g = hptr[h]; g < hptr[h + 1]; ++g) {
            maxne[h] = std::max(maxne[h], ne[g]);
            maxm[h] = std::max(maxm[h], m[g]);
        }
        for (int s = 0; s < 2; ++s)
            for (int c : kids[s][h]) maxnb[h] = std::max(maxnb[h], m[c] - ne[c]);
        const int nq = (maxne[h] + w - 1) / w;
        trail_tiles[h].assign(nq, 0);
        panel_rows[h].assign(nq, 0);
        for (int g = hptr[h]; g < hptr[h + 1]; ++g) {
            for (int q = 0; q < nq; ++q) {
                trail_tiles[h][q] = std::max(trail_tiles[h][q], syrk_tiles(false, q * w, ne[g], ld[g]));
                panel_rows[h][q] = std::max(panel_rows[h][q], panel_rowblocks(q * w, ne[g], ld[g]));
            }
            schur_tiles[h] = std::max(schur_tiles[h], syrk_tiles(true, 0, ne[g], m[g]));
        }
    }
    return "";
}

std::string CoarseSolver::alloc(void* (*alloc_fn)(void*, size_t), void* ctx, hipStream_t s) {
    auto A = [&](size_t bytes) { return alloc_fn(ctx, bytes ? bytes : 8); };
    bool ok = true;
    auto up = [&](const auto& v, auto*& d) {
        using V = typename std::decay<decltype(v)>::type::value_type;
        d = (std::remove_reference_t<decltype(d)>)A(v.size() * sizeof(V));
        if (!d) { ok = false; return; }
        if (!v.empty()) ok = ok && hipMemcpy(d, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice) == hipSuccess;
    };
    F = (double*)A(nF * sizeof(double));
    z = (double*)A(nZ * sizeof(double));
    z2 = (double*)A(nZ * sizeof(double));
    Wbuf = (double*)A((size_t)maxnf * panel_wbuf_stride() * sizeof(double));
    info = (int*)A((size_t)(1 + maxnf) * sizeof(int));
    if (!F || !z || !z2 || !Wbuf || !info) return "device allocation failed (coarse fronts)";
    up(foff, d_foff); up(zoff, d_zoff); up(pmoff, d_pmoff);
    up(ne, d_ne); up(m, d_m); up(ld, d_ld); up(parent, d_parent); up(vars, d_vars); up(pmap, d_pmap);
    up(sub_pos, d_sub_pos); up(sub_front, d_sub_front);
    for (int sl = 0; sl < 2; ++sl) {
        d_kids[sl].assign(H, nullptr);
        for (int h = 0; h < H; ++h)
            if (!kids[sl][h].empty()) up(kids[sl][h], d_kids[sl][h]);
    }
    (void)s;
    return ok ? "" : "device allocation or upload failed (coarse structure)";
}

// ------------------------------------------------------------------ numeric
void CoarseSolver::factor(hipStream_t s, const int* color_list, const std::vector<int>& color_ptr,
                          const int* nPv, const double* Sp, int sp_stride) {
    hipMemsetAsync(F, 0, nF * sizeof(double), s);
    hipMemsetAsync(info, 0, (size_t)(1 + maxnf) * sizeof(int), s);
    const int w = interior_panel_width();
    for (int h = 0; h < H; ++h) {
        const int f0 = hptr[h], nf = hptr[h + 1] - hptr[h];
        if (h == 0) {
            for (size_t c = 0; c + 1 < color_ptr.size(); ++c) {
                const int cnt = color_ptr[c + 1] - color_ptr[c];
                if (cnt == 0) continue;
                hipLaunchKernelGGL(k_nd_leaf_assemble, dim3(cnt), dim3(256), 0, s, color_list + color_ptr[c], nPv, Sp,
                                   sp_stride, d_sub_pos, maxp, d_sub_front, d_foff, d_ld, F);
            }
        } else {
            for (int sl = 0; sl < 2; ++sl) {
                const int nk = (int)kids[sl][h].size();
                if (nk == 0 || maxnb[h] == 0) continue;
                hipLaunchKernelGGL(k_nd_extend, dim3(maxnb[h], nk), dim3(256), 0, s, d_kids[sl][h], d_parent, d_foff,
                                   d_ne, d_m, d_ld, d_pmoff, d_pmap, F);
            }
        }
        if (pin_front >= f0 && pin_front < f0 + nf)
            hipLaunchKernelGGL(k_nd_set_one, dim3(1), dim3(1), 0, s, F,
                               foff[pin_front] + (int64_t)pin_pos * (ld[pin_front] + 1));
        if (maxne[h] > 0)
            hipLaunchKernelGGL(k_nd_eye, dim3(nb(maxne[h], 256), nf), dim3(256), 0, s, d_foff + f0, d_ne + f0,
                               d_m + f0, d_ld + f0, F);
        // panels and trailing updates over all rows (boundary and X rows);
        // the Schur update only over the boundary block
        const int nq = (int)trail_tiles[h].size();
        for (int q = 0; q < nq; ++q) {
            launch_interior_panel<double>(s, nf, F, d_foff + f0, d_ld + f0, d_ne + f0, d_ld + f0, q * w, Wbuf,
                                          panel_rows[h][q], info + 1);
            launch_syrk_update<double>(s, nf, F, d_foff + f0, d_ld + f0, d_ne + f0, d_ld + f0, false, q * w,
                                       trail_tiles[h][q]);
        }
        launch_syrk_update<double>(s, nf, F, d_foff + f0, d_ld + f0, d_ne + f0, d_m + f0, true, 0, schur_tiles[h]);
    }
    hipLaunchKernelGGL(k_nd_info, dim3(1), dim3(256), 0, s, maxnf, info + 1, info);
}

void CoarseSolver::solve(hipStream_t s, double* b) {
    for (int h = 0; h < H; ++h) {
        const int f0 = hptr[h], nf = hptr[h + 1] - hptr[h];
        hipLaunchKernelGGL(k_nd_gather_e, dim3(nb(std::max(maxm[h], 1), 256), nf), dim3(256), 0, s, d_zoff + f0,
                           d_ne + f0, d_m + f0, d_vars, b, z);
        for (int sl = 0; sl < 2 && h > 0; ++sl) {
            const int nk = (int)kids[sl][h].size();
            if (nk == 0 || maxnb[h] == 0) continue;
            hipLaunchKernelGGL(k_nd_extend_vec, dim3(nb(maxnb[h], 256), nk), dim3(256), 0, s, d_kids[sl][h],
                               d_parent, d_zoff, d_ne, d_m, d_pmoff, d_pmap, z);
        }
        if (maxne[h] == 0) continue;
        // y = X^T z_e (into z2), then z_b -= L_be y
        hipLaunchKernelGGL(k_nd_gemv_t, dim3(nb(maxne[h], 4), nf), dim3(256), 0, s, d_foff + f0, d_ne + f0, d_m + f0,
                           d_ld + f0, 0, F, d_zoff + f0, z, nullptr, z2, 1.0);
        if (maxm[h] > 0)
            hipLaunchKernelGGL(k_nd_gemv_n, dim3(nb(maxm[h], GN_RB), nf), dim3(256), 0, s, d_foff + f0, d_ne + f0,
                               d_m + f0, d_ld + f0, 1, F, d_zoff + f0, z2, z, z, -1.0);
    }
    for (int h = H - 1; h >= 0; --h) {
        const int f0 = hptr[h], nf = hptr[h + 1] - hptr[h];
        if (maxne[h] == 0) continue;
        // z_b = x_b; t = y - L_be^T x_b (into z_e); x_e = X t (into z2)
        hipLaunchKernelGGL(k_nd_gather_b, dim3(nb(std::max(maxm[h], 1), 256), nf), dim3(256), 0, s, d_zoff + f0,
                           d_ne + f0, d_m + f0, d_vars, b, z);
        hipLaunchKernelGGL(k_nd_gemv_t, dim3(nb(maxne[h], 4), nf), dim3(256), 0, s, d_foff + f0, d_ne + f0, d_m + f0,
                           d_ld + f0, 1, F, d_zoff + f0, z, z2, z, -1.0);
        hipLaunchKernelGGL(k_nd_gemv_n, dim3(nb(maxne[h], GN_RB), nf), dim3(256), 0, s, d_foff + f0, d_ne + f0, d_m + f0,
                           d_ld + f0, 0, F, d_zoff + f0, z, nullptr, z2, 1.0);
        hipLaunchKernelGGL(k_nd_scatter_e, dim3(nb(maxne[h], 256), nf), dim3(256), 0, s, d_zoff + f0, d_ne + f0,
                           d_vars, z2, b);
    }
}

}  // namespace bdm
