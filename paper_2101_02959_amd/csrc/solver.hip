// Host-side control of the Newton-Krylov BDDC / FETI-DP deluxe time step
// (paper Sec. 3b-c, 4, 6).  Every numerical step runs in the HIP kernels of
// fe.hip, dense.hip, bddc.hip and vec.hip; this file builds the index maps,
// owns the device workspace and sequences the launches.
#include "solver.hpp"
#include "pcg_slots.hpp"

#include <algorithm>
#include <functional>
#include <chrono>
#include <limits>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <cstdlib>

namespace bdm {

namespace {
thread_local std::string g_err;


// Device allocation recorded in the context list c (freed with the context).
static void* ctx_alloc(void* c, size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 8) != hipSuccess) return nullptr;
    static_cast<std::vector<void*>*>(c)->push_back(p);
    return p;
}
constexpr int MAXOBJ = 1280;   // largest face / edge (dofs): H/h up to 26

template <typename T>
__global__ void k_sub_t(int64_t n, const T* __restrict__ x, T* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] -= x[i];
}

__global__ void k_lin_comb(int64_t n, double a, const double* __restrict__ x, double b,
                           const double* __restrict__ y, double* __restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = a * x[i] + b * y[i];
}

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Extreme eigenvalues of the symmetric tridiagonal Lanczos matrix by
// bisection on Sturm sequences.
double sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
    int cnt = 0;
    double q = 1.0;
    for (size_t i = 0; i < d.size(); ++i) {
        const double off = (i == 0) ? 0.0 : e[i - 1] * e[i - 1];
        q = d[i] - x - (i == 0 ? 0.0 : off / (q == 0.0 ? 1e-300 : q));
        if (q < 0) ++cnt;
    }
    return cnt;
}
double tri_eig(const std::vector<double>& d, const std::vector<double>& e, int k) {
    double lo = 1e300, hi = -1e300;
    for (size_t i = 0; i < d.size(); ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0) + (i + 1 < d.size() ? std::fabs(e[i]) : 0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(d, e, mid) > k) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}
double lanczos_cond(const std::vector<double>& a, const std::vector<double>& b) {
    const size_t k = a.size();
    if (k == 0) return 1.0;
    std::vector<double> d(k), e(k > 0 ? k - 1 : 0);
    for (size_t i = 0; i < k; ++i) {
        d[i] = 1.0 / a[i] + (i > 0 ? b[i - 1] / a[i - 1] : 0.0);
        if (i + 1 < k) e[i] = std::sqrt(std::max(b[i], 0.0)) / a[i];
    }
    const double lmin = tri_eig(d, e, 0), lmax = tri_eig(d, e, (int)k - 1);
    return lmax / lmin;
}

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

#define HIPOK(x)                                                                      \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x); \
            return BDM_E_HIP;                                                         \
        }                                                                             \
    } while (0)

Context::~Context() {
    for (auto& g : kry_exec_)
        if (g) hipGraphExecDestroy(g);
    if (kry_stream_) hipStreamDestroy(kry_stream_);
    if (side_stream_) hipStreamDestroy(side_stream_);
    if (ev_fork_) hipEventDestroy(ev_fork_);
    if (ev_join_) hipEventDestroy(ev_join_);
    if (ev_free_) hipEventDestroy(ev_free_);
    if (ev_ready_) hipEventDestroy(ev_ready_);
    for (void* p : allocs_) hipFree(p);
}

void* Context::dalloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 8;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    allocs_.push_back(p);
    return p;
}

template <typename V>
V* Context::upload(const std::vector<V>& h) {
    V* d = (V*)dalloc(h.size() * sizeof(V));
    if (d && !h.empty()) hipMemcpy(d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice);
    return d;
}

int Context::sync() {
    HIPOK(hipStreamSynchronize(stream_));
    return 0;
}

// x . y read back to the host (a synchronisation).  A HIP failure sets
// hip_err_ and the message and returns NaN, which every caller treats as a
// failed step; callers return BDM_E_HIP when hip_err_ is set.
double Context::dot(int64_t n, const double* x, const double* y) {
    launch_dot(stream_, n, x, y, part_, tick_, scal_);
    double h = 0.0;
    hipError_t e = hipMemcpyAsync(&h, scal_, sizeof(double), hipMemcpyDeviceToHost, stream_);
    if (e == hipSuccess) e = hipStreamSynchronize(stream_);
    if (e != hipSuccess) {
        hip_err_ = true;
        set_error(std::string("HIP error in a reduction: ") + hipGetErrorString(e));
        return std::numeric_limits<double>::quiet_NaN();
    }
    return h;
}

int Context::create(const bdm_mesh* m, const bdm_physics* ph, const bdm_opts* o, hipStream_t s) {
    stream_ = s;
    opts = *o;
    phys = *ph;
    // The Dirichlet solves run as one fused forward/backward launch unless
    // BDM_DIRICHLET_FUSED=0 (the same arithmetic either way).
    if (const char* e = std::getenv("BDM_DIRICHLET_FUSED")) fused_dirichlet_ = std::atoi(e) != 0;
    if (const char* e = std::getenv("BDM_SETUP_OVERLAP")) setup_overlap_ = std::atoi(e) != 0;
    if (!(o->dt > 0) || o->newton_maxit < 1 || o->krylov_maxit < 1 ||
        (o->schedule != BDM_SCHED_QUEUE && o->schedule != BDM_SCHED_GRID) ||
        (o->krylov_reduced != 0 && o->krylov_reduced != 1) ||
        (o->scaling != BDM_SCALING_DELUXE && o->scaling != BDM_SCALING_RHO) ||
        (o->primal != BDM_PRIMAL_VE && o->primal != BDM_PRIMAL_V && o->primal != BDM_PRIMAL_VEF)) {
        set_error("invalid options");
        return BDM_E_ARG;
    }
    const bool mapped = m->geometry == BDM_GEOM_ELLIPSOID;
    if (m->geometry != BDM_GEOM_BOX && !mapped) {
        set_error("unknown mesh geometry");
        return BDM_E_ARG;
    }
    if (mapped) {
        const double* g = m->ellipsoid;
        const double hpi = 0.5 * M_PI;
        bool ok = true;
        for (int q = 0; q < 10; ++q) ok = ok && std::isfinite(g[q]);
        ok = ok && 0.0 < g[0] && g[0] < g[1] && 0.0 < g[2] && g[2] < g[3] && 0.0 < g[4] && g[4] < g[5];
        ok = ok && -hpi < g[6] && g[6] < g[7] && g[7] < hpi && g[8] < g[9] && g[9] <= g[8] + 2.0 * M_PI;
        if (!ok) {
            set_error("ellipsoid parameters need 0 < a1 < a2, 0 < b1 < b2, 0 < c1 < c2, "
                      "-pi/2 < theta_min < theta_max < pi/2 and phi_min < phi_max <= phi_min + 2 pi");
            return BDM_E_ARG;
        }
    }
    // the element size is unused on a mapped mesh
    std::string err = topo.build(m->nx, m->ny, m->nz, mapped ? 1.0 : m->h, m->px, m->py, m->pz, m->cuts_x,
                                 m->cuts_y, m->cuts_z, o->primal);
    if (!err.empty()) {
        set_error(err);
        return BDM_E_ARG;
    }
    prec_ = (o->precision == BDM_PREC_MIXED) ? 1 : 0;
    tsize_ = prec_ ? sizeof(float) : sizeof(double);
    N = topo.N;
    fp.nx = m->nx; fp.ny = m->ny; fp.nz = m->nz;
    fp.nx1 = m->nx + 1; fp.ny1 = m->ny + 1;
    fp.N = N;
    fp.h = m->h; fp.tau = o->dt; fp.c = ph->chi * ph->Cm;
    fp.hy = m->hy > 0.0 ? m->hy : m->h;
    fp.hz = m->hz > 0.0 ? m->hz : m->h;
    fp.chiG = ph->chi * ph->G; fp.chieta1 = ph->chi * ph->eta1; fp.eta2 = ph->eta2;
    fp.vth = ph->vth; fp.vp = ph->vp;

    if (!mapped) {
        const double hd[3] = {fp.h, fp.hy, fp.hz};
        std::vector<double> ke = layer_matrices(m->nz, hd, o->dt, ph->sigma_i, ph->sigma_e, ph->theta0, ph->theta1);
        std::vector<double> st = stencil_tables(m->nz, ke);
        ke_ = upload(ke);
        st_ = upload(st);
    }

    const int nsub = (int)topo.subs.size();
    // ---------------- per-subdomain descriptors
    std::vector<int> n(nsub), nI(nsub), nr(nsub), nV(nsub), nc(nsub), nP(nsub), box(6 * nsub), kF(nsub);
    std::vector<int64_t> lmap_off(nsub), K_off(nsub), F_off(nsub), Z_off(nsub), P_off(nsub);
    std::vector<int64_t> xI_off(nsub), xr_off(nsub), LII(nsub), Lrr(nsub), Srr_off(nsub);
    std::vector<int> lmap, primal, Ilist;
    std::vector<int> st1c0(nsub, 0), st1c1(nsub), st1c2(nsub), st2c1(nsub), nIcv(nsub);
    int64_t accK = 0, accF = 0, accZ = 0, accP = 0, accI = 0, accR = 0, accS = 0, accLII = 0, accLrr = 0;
    for (int q = 0; q < nsub; ++q) {
        const SubInfo& sb = topo.subs[q];
        if (sb.nc > MAXC || sb.nV > MAXV) {
            set_error("subdomain has too many primal constraints");
            return BDM_E_ARG;
        }
        n[q] = sb.n(); nI[q] = sb.nI; nr[q] = sb.nr; nV[q] = sb.nV; nc[q] = sb.nc; nP[q] = sb.nP;
        nIcv[q] = sb.nIc;
        kF[q] = sb.nc + sb.nV;
        box[6 * q + 0] = sb.ex0; box[6 * q + 1] = sb.ey0; box[6 * q + 2] = sb.ez0;
        box[6 * q + 3] = sb.Lx(); box[6 * q + 4] = sb.Ly(); box[6 * q + 5] = sb.Lz();
        maxbox_ = std::max(maxbox_, (sb.Lx() + 1) * (sb.Ly() + 1) * (sb.Lz() + 1));
        maxG_ = std::max(maxG_, sb.n() - sb.nI);
        maxnI_ = std::max(maxnI_, sb.nI);
        maxn_ = std::max(maxn_, sb.n());
        maxnr_ = std::max(maxnr_, sb.nr);
        lmap_off[q] = (int64_t)lmap.size();
        lmap.insert(lmap.end(), sb.lmap.begin(), sb.lmap.end());
        K_off[q] = accK; accK += (int64_t)sb.n() * sb.n();
        LII[q] = accLII; accLII += pp_size(sb.nI);
        Lrr[q] = accLrr; accLrr += pp_size(sb.nr);
        F_off[q] = accF; accF += (int64_t)sb.nr * (sb.nc + sb.nV);
        Z_off[q] = accZ; accZ += (int64_t)sb.nr * sb.nP;
        P_off[q] = accP; accP += sb.nP;
        primal.insert(primal.end(), sb.primal.begin(), sb.primal.end());
        xI_off[q] = accI; accI += sb.nI;
        Ilist.insert(Ilist.end(), sb.I_nodes.begin(), sb.I_nodes.end());
        xr_off[q] = accR; accR += sb.nr;
        Srr_off[q] = accS; accS += (int64_t)sb.nr * sb.nr;
        st1c1[q] = sb.nI; st1c2[q] = sb.n(); st2c1[q] = sb.nI + sb.nr;
    }
    nK_ = accK; nF_ = accF; nZ_ = accZ; nxI_ = accI; nxr_ = accR; nSrr_ = accS;
    nLII_ = accLII; nLrr_ = accLrr;
    // chunks of subdomains whose local matrices fit the setup workspace
    {
        double gb = 16.0;
        if (const char* e = std::getenv("BDM_SETUP_WORKSPACE_GB")) gb = std::atof(e);
        const int64_t budget = std::max<int64_t>((int64_t)(gb * 1e9) / (int64_t)tsize_, 1);
        std::vector<int64_t> kc(nsub);
        int64_t total = 0, maxsz = 0;
        for (int q = 0; q < nsub; ++q) {
            total += (int64_t)n[q] * n[q];
            maxsz = std::max<int64_t>(maxsz, (int64_t)n[q] * n[q]);
        }
        // equal subdomain counts per chunk, as many chunks as the budget needs
        int nch = (int)std::max<int64_t>(1, (total + budget - 1) / budget);
        for (;;) {
            const int per = (nsub + nch - 1) / nch;
            int64_t worst = 0;
            for (int c0 = 0; c0 < nsub; c0 += per) {
                int64_t acc = 0;
                for (int q = c0; q < std::min(nsub, c0 + per); ++q) acc += (int64_t)n[q] * n[q];
                worst = std::max(worst, acc);
            }
            if (worst <= budget || per == 1) break;
            ++nch;
        }
        const int per = (nsub + nch - 1) / nch;
        chunks_.clear();
        for (int c0 = 0; c0 < nsub; c0 += per) {
            const int c1 = std::min(nsub, c0 + per);
            chunks_.push_back({c0, c1});
            int64_t acc = 0;
            for (int q = c0; q < c1; ++q) {
                kc[q] = acc;
                acc += (int64_t)n[q] * n[q];
            }
            nKwork_ = std::max(nKwork_, acc);
        }
        (void)maxsz;
        Kc_off_ = upload(kc);
        // elimination plans (launch sizes: tiles per matrix, max over the batch):
        // the interior block with the Schur update, and the r-block of S_Gamma
        // viewed as its own matrix at offset (nI, nI)
        std::vector<int64_t> kr(nsub);
        for (int q = 0; q < nsub; ++q) kr[q] = kc[q] + (int64_t)nI[q] + (int64_t)nI[q] * n[q];
        plan_int_.off = Kc_off_;
        plan_int_.nIc = upload(nIcv);
        plan_rr_.off = upload(kr);
        build_plan(plan_int_, true, 0);
        build_plan(plan_rr_, false, 0);
    }
    nInodes_ = (int)Ilist.size();

    // ---------------- objects (faces then edges) and their shares
    const int nF = (int)topo.faces.size(), nE = (int)topo.edges.size();
    const int nobj = nF + nE;
    std::vector<int> on(nobj), onodes, sh_ptr(nobj + 1, 0), sh_sub, sh_roff;
    std::vector<int64_t> onode_off(nobj), ofac(nobj), sh_slot, sh_yoff;
    std::map<std::pair<int, int>, int64_t> slot_of;   // (object, sub) -> slot offset
    std::map<std::pair<int, int>, int> roff_of;       // (object, sub) -> r offset
    for (int q = 0; q < nsub; ++q) {
        const SubInfo& sb = topo.subs[q];
        for (size_t t = 0; t < sb.faces.size(); ++t) roff_of[{sb.faces[t], q}] = sb.face_off[t];
        for (size_t t = 0; t < sb.edges.size(); ++t) roff_of[{nF + sb.edges[t], q}] = sb.edge_off[t];
    }
    int64_t accSlot = 0, accFac = 0, accY = 0;
    nface_obj_ = nF;
    for (int ob = 0; ob < nobj; ++ob) {
        const Object& O = ob < nF ? topo.faces[ob] : topo.edges[ob - nF];
        on[ob] = 2 * (int)O.nodes.size();
        maxobjn_ = std::max(maxobjn_, on[ob]);
        if (ob < nF) maxface_n_ = std::max(maxface_n_, on[ob]);
        else maxedge_n_ = std::max(maxedge_n_, on[ob]);
        if (on[ob] > MAXOBJ || (int)O.subs.size() > deluxe_max_shares()) {
            set_error("interface object larger or more widely shared than supported");
            return BDM_E_ARG;
        }
        onode_off[ob] = (int64_t)onodes.size();
        onodes.insert(onodes.end(), O.nodes.begin(), O.nodes.end());
        ofac[ob] = accFac; accFac += (int64_t)on[ob] * on[ob];
        for (int sbi : O.subs) {
            slot_of[{ob, sbi}] = accSlot;
            sh_sub.push_back(sbi);
            sh_roff.push_back(roff_of.at({ob, sbi}));
            sh_slot.push_back(accSlot);
            sh_yoff.push_back(accY);
            accSlot += (int64_t)on[ob] * on[ob];
            accY += on[ob];
        }
        sh_ptr[ob + 1] = (int)sh_sub.size();
    }
    nslot_ = accSlot; nfac_ = accFac; nyb_ = accY;
    // rho scaling weights (Sec. 4.2): share m of an object gets
    // sigma_M^(m) / sum_k sigma_M^(k) per field, sigma_M the largest principal
    // conductivity (sigma^i for v, sigma^e for u_e).  The tissue parameters
    // are the same in every subdomain, so each weight is 1 / (shares).
    std::vector<double> rho_w(2 * sh_sub.size());
    {
        const double sMi = std::max({phys.sigma_i[0], phys.sigma_i[1], phys.sigma_i[2]});
        const double sMe = std::max({phys.sigma_e[0], phys.sigma_e[1], phys.sigma_e[2]});
        for (int ob = 0; ob < nobj; ++ob) {
            const int nsh = sh_ptr[ob + 1] - sh_ptr[ob];
            for (int q = sh_ptr[ob]; q < sh_ptr[ob + 1]; ++q) {
                rho_w[2 * q] = sMi / (nsh * sMi);
                rho_w[2 * q + 1] = sMe / (nsh * sMe);
            }
        }
    }
    if (maxobjn_ > deluxe_max_object()) {
        set_error("a face or edge has more than " + std::to_string(deluxe_max_object()) + " dofs");
        return BDM_E_ARG;
    }
    {
        // the per-iteration triangular solves keep a subdomain's vector in LDS
        int dev = 0, lds = 0;
        HIPOK(hipGetDevice(&dev));
        HIPOK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const int64_t need = (int64_t)std::max(maxnI_, maxnr_) * (int64_t)tsize_;
        if (need > lds) {
            set_error("a subdomain has " + std::to_string(std::max(maxnI_, maxnr_)) + " interior or interface dofs; " +
                      "its triangular-solve vector (" + std::to_string(need) + " bytes) exceeds the " +
                      std::to_string(lds) + " bytes of LDS per workgroup (FP32 local factors halve it)");
            return BDM_E_ARG;
        }
    }
    // per-subdomain object lists
    std::vector<int64_t> so_ptr(nsub + 1, 0), so_slot;
    std::vector<int> so_roff, so_n, so_kind, so_nnode, so_eidx;
    for (int q = 0; q < nsub; ++q) {
        const SubInfo& sb = topo.subs[q];
        for (size_t t = 0; t < sb.faces.size(); ++t) {
            const int ob = sb.faces[t];
            so_roff.push_back(sb.face_off[t]); so_n.push_back(on[ob]);
            so_slot.push_back(slot_of.at({ob, q})); so_kind.push_back(0);
            so_nnode.push_back(on[ob] / 2); so_eidx.push_back(sb.face_con[t]);
        }
        for (size_t t = 0; t < sb.edges.size(); ++t) {
            const int ob = nF + sb.edges[t];
            so_roff.push_back(sb.edge_off[t]); so_n.push_back(on[ob]);
            so_slot.push_back(slot_of.at({ob, q})); so_kind.push_back(1);
            so_nnode.push_back(on[ob] / 2); so_eidx.push_back(sb.edge_con[t]);
        }
        so_ptr[q + 1] = (int64_t)so_roff.size();
    }
    // FETI-DP pairs
    std::vector<int> pr_ptr(nobj + 1, 0), pr_a, pr_b, pr_qa, pr_qb;
    std::vector<int64_t> pr_off;
    int64_t accL = 0;
    for (int ob = 0; ob < nobj; ++ob) {
        const int b0 = sh_ptr[ob], b1 = sh_ptr[ob + 1];
        for (int qa = b0; qa < b1; ++qa)
            for (int qb = qa + 1; qb < b1; ++qb) {
                pr_a.push_back(sh_sub[qa]); pr_b.push_back(sh_sub[qb]);
                pr_qa.push_back(qa); pr_qb.push_back(qb);
                pr_off.push_back(accL);
                accL += on[ob];
            }
        pr_ptr[ob + 1] = (int)pr_a.size();
    }
    nlam_ = (long)accL;
    // coarse gather lists
    const int np = topo.nprimal;
    std::vector<std::vector<std::pair<int, int>>> contrib(np);
    for (int q = 0; q < nsub; ++q)
        for (int a = 0; a < topo.subs[q].nP; ++a) contrib[topo.subs[q].primal[a]].push_back({q, a});
    std::vector<int> cp_ptr(np + 1, 0), cp_sub, cp_loc, vnode;
    for (int p = 0; p < np; ++p) {
        for (auto& c : contrib[p]) { cp_sub.push_back(c.first); cp_loc.push_back(c.second); }
        cp_ptr[p + 1] = (int)cp_sub.size();
    }
    for (auto& vo : topo.verts) vnode.push_back(vo.nodes[0]);
    // colours of the subdomain grid (same colour => no shared primal object)
    colors_.assign(8, {});
    for (int q = 0; q < nsub; ++q) {
        const SubInfo& sb = topo.subs[q];
        colors_[(sb.a & 1) + 2 * (sb.b & 1) + 4 * (sb.c & 1)].push_back(q);
    }
    std::vector<int> clist;
    color_ptr_.assign(1, 0);
    for (auto& c : colors_) {
        clist.insert(clist.end(), c.begin(), c.end());
        color_ptr_.push_back((int)clist.size());
    }

    // ---------------- upload descriptors
    bd_.nsub = nsub;
    bd_.sub0 = 0;
    bd_.n = upload(n); bd_.nI = upload(nI); bd_.nr = upload(nr); bd_.nV = upload(nV); bd_.nc = upload(nc);
    bd_.K_off = Kc_off_; bd_.box = upload(box); bd_.lmap_off = upload(lmap_off); bd_.lmap = upload(lmap);
    bd_.F_off = upload(F_off); bd_.Z_off = upload(Z_off);
    bd_.so_ptr = upload(so_ptr); bd_.so_roff = upload(so_roff); bd_.so_n = upload(so_n);
    bd_.so_slot = upload(so_slot); bd_.so_kind = upload(so_kind); bd_.so_nnode = upload(so_nnode);
    bd_.so_eidx = upload(so_eidx); bd_.Srr_off = upload(Srr_off);
    od_.nobj = nobj; od_.maxn = maxobjn_; od_.n = upload(on); od_.node_off = upload(onode_off); od_.nodes = upload(onodes);
    od_.fac_off = upload(ofac); od_.sh_ptr = upload(sh_ptr); od_.sh_sub = upload(sh_sub);
    od_.sh_roff = upload(sh_roff); od_.sh_slot = upload(sh_slot);
    sv_.nsub = nsub; sv_.nr = bd_.nr; sv_.nV = bd_.nV; sv_.nc = bd_.nc;
    xr_off_ = upload(xr_off); sv_.xoff = xr_off_; sv_.F_off = bd_.F_off; sv_.Z_off = bd_.Z_off;
    sv_.P_off = upload(P_off); sv_.primal = upload(primal);
    cd_.np = np; cd_.nverts = (int)topo.verts.size(); cd_.vnode = upload(vnode);
    cd_.cp_ptr = upload(cp_ptr); cd_.cp_sub = upload(cp_sub); cd_.cp_loc = upload(cp_loc);
    fd_.pr_ptr = upload(pr_ptr); fd_.pr_a = upload(pr_a); fd_.pr_b = upload(pr_b);
    fd_.pr_qa = upload(pr_qa); fd_.pr_qb = upload(pr_qb); fd_.pr_off = upload(pr_off);
    fd_.sh_yoff = upload(sh_yoff);
    rho_w_ = upload(rho_w);
    Ilist_ = upload(Ilist);
    LII_off_ = upload(LII); Lrr_off_ = upload(Lrr); xI_off_ = upload(xI_off); Srr_off_ = bd_.Srr_off;
    nI_ = bd_.nI; nr_ = bd_.nr; ld_ = bd_.n; kF_ = upload(kF); nP_ = upload(nP);
    // work queues of the per-iteration triangular solves: subdomains in
    // decreasing factor size (cost n^2), longest first
    if (opts.schedule == BDM_SCHED_QUEUE) {
        auto lpt = [&](const std::vector<int>& sz) {
            std::vector<int> o(nsub);
            for (int q = 0; q < nsub; ++q) o[q] = q;
            std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return sz[a] > sz[b]; });
            return o;
        };
        qctr_ = (int*)dalloc(2 * sizeof(int));
        if (!qctr_) {
            set_error("device allocation failed (work queue)");
            return BDM_E_OOM;
        }
        HIPOK(hipMemsetAsync(qctr_, 0, 2 * sizeof(int), stream_));
        qI_.order = upload(lpt(nI));
        qI_.counter = qctr_;
        qr_.order = upload(lpt(nr));
        qr_.counter = qctr_;
    }
    st1c0_ = upload(st1c0); st1c1_ = upload(st1c1); st1c2_ = upload(st1c2); st2c1_ = upload(st2c1);
    plan_int_.ne = st1c1_; plan_int_.n = st1c2_;
    plan_rr_.ne = nr_; plan_rr_.n = nr_;
    color_list_ = upload(clist);
    std::vector<int64_t> z64(1, 0);
    std::vector<int> zi(1, 0), npv(1, np);
    zero64_ = upload(z64); cpin_ = upload(zi); np_ = upload(npv);
    one_ = upload(npv);
    // pin: the u_e dof of the first vertex (every primal space has vertices)
    pin_ = 1;
    // coarse problem: nested dissection of the subdomain grid
    {
        const std::string e = coarse_.init(topo, pin_, MAXP);
        if (!e.empty()) {
            set_error(e);
            return BDM_E_ARG;
        }
    }

    // ---------------- global vectors and workspace
    const size_t vb = (size_t)N * sizeof(double);
    v_ = (double*)dalloc(vb); ue_ = (double*)dalloc(vb); w_ = (double*)dalloc(vb); vn_ = (double*)dalloc(vb);
    vprev_ = (double*)dalloc(vb); ueprev_ = (double*)dalloc(vb); Is_ = (double*)dalloc(vb);
    dg_ = (double*)dalloc(vb); vlin_ = (double*)dalloc(vb); wlin_ = (double*)dalloc(vb);
    bad_ = (int*)dalloc(sizeof(int));
    const size_t kb = (size_t)std::max<int64_t>(2 * N, nlam_ + 2 * N) * sizeof(double);
    kx_ = (double*)dalloc(kb); kr_ = (double*)dalloc(kb); kz_ = (double*)dalloc(kb);
    kp_ = (double*)dalloc(kb); kq_ = (double*)dalloc(kb);
    t1_ = (double*)dalloc(2 * vb); t2_ = (double*)dalloc(2 * vb); t3_ = (double*)dalloc(2 * vb);
    gzero_ = (double*)dalloc(2 * vb);
    R_ = (double*)dalloc(2 * vb); S_ = (double*)dalloc(2 * vb); U_ = (double*)dalloc(2 * vb);
    Rt_ = (double*)dalloc(2 * vb);
    part_ = (double*)dalloc(dot_partials() * sizeof(double));
    scal_ = (double*)dalloc(8 * sizeof(double));
    tick_ = (unsigned*)dalloc(vec_tickets() * sizeof(unsigned));
    if (!tick_ || hipMemset(tick_, 0, vec_tickets() * sizeof(unsigned)) != hipSuccess) {
        set_error("device allocation failed (reduction tickets)");
        return BDM_E_OOM;
    }
    kry_hcap_ = std::max(opts.krylov_maxit, 1) + 1;
    kry_sc_ = (double*)dalloc(PCG_NSLOT * sizeof(double));
    kry_hist_ = (double*)dalloc((kry_hcap_ + 1) * sizeof(double));
    kry_ah_ = (double*)dalloc(kry_hcap_ * sizeof(double));
    kry_bh_ = (double*)dalloc(kry_hcap_ * sizeof(double));
    if (!kry_sc_ || !kry_hist_ || !kry_ah_ || !kry_bh_) {
        set_error("device allocation failed (Krylov history)");
        return BDM_E_OOM;
    }
    if (!v_ || !ue_ || !w_ || !kx_ || !R_ || !Rt_ || !part_ || !scal_) {
        set_error("device allocation failed (global vectors)");
        return BDM_E_OOM;
    }
    HIPOK(hipMemsetAsync(gzero_, 0, 2 * vb, stream_));
    if (mapped) {
        // isoparametric element matrices, per-node stencils and masses of the
        // ellipsoid, built on the device
        const int64_t ne = (int64_t)m->nx * m->ny * m->nz;
        double* ke = (double*)dalloc((size_t)ne * 128 * sizeof(double));
        double* mec = (double*)dalloc((size_t)ne * 8 * sizeof(double));
        double* stn = (double*)dalloc((size_t)N * 54 * sizeof(double));
        double* mnode = (double*)dalloc(vb);
        if (!ke || !mec || !stn || !mnode || !bad_) {
            set_error("device allocation failed (mapped mesh)");
            return BDM_E_OOM;
        }
        EllGeom g;
        for (int q = 0; q < 10; ++q) g.p[q] = m->ellipsoid[q];
        IsoMedia md;
        for (int q = 0; q < 3; ++q) {
            md.sig_i[q] = ph->sigma_i[q];
            md.sig_e[q] = ph->sigma_e[q];
        }
        md.th0 = ph->theta0; md.th1 = ph->theta1; md.tau = o->dt;
        HIPOK(hipMemsetAsync(bad_, 0, sizeof(int), stream_));
        launch_mapped_mesh(stream_, fp, g, md, ke, mec, stn, mnode, bad_);
        HIPOK(hipGetLastError());
        int hb = 0;
        HIPOK(hipMemcpyAsync(&hb, bad_, sizeof(int), hipMemcpyDeviceToHost, stream_));
        HIPOK(hipStreamSynchronize(stream_));
        if (hb) {
            set_error("an ellipsoid element has a non-positive Jacobian determinant");
            return BDM_E_ARG;
        }
        ke_ = ke;
        fp.mec = mec; fp.stn = stn; fp.mnode = mnode;
    }
    int rc = prec_ ? alloc_local<float>() : alloc_local<double>();
    if (rc) return rc;
    // autotuner: device name, optional JSON cache, stencil tile shape
    {
        int dev = 0;
        hipDeviceProp_t prop;
        HIPOK(hipGetDevice(&dev));
        HIPOK(hipGetDeviceProperties(&prop, dev));
        tuner_.device = prop.gcnArchName;
        if (const char* e = std::getenv("BDM_TUNE_CACHE")) tune_path_ = e;
        if (!tune_path_.empty()) {
            const std::string err = tuner_.load(tune_path_);
            if (!err.empty()) {
                set_error(err + " (" + tune_path_ + ")");
                return BDM_E_ARG;
            }
        }
        if (!fp.stn && (rc = tune_stencil())) return rc;   // mapped meshes have one stencil kernel
        if ((rc = save_tuning())) return rc;
    }
    return set_state(nullptr, nullptr, nullptr, 0.0, false);
}

template <typename T>
int Context::alloc_local() {
    const int nsub = (int)topo.subs.size();
    const bool feti = opts.solver == BDM_SOLVER_FETIDP;
    K_ = dalloc(nKwork_ * sizeof(T));
    {
        int maxc = 1;
        for (const auto& ch : chunks_) maxc = std::max(maxc, ch.second - ch.first);
        Wbuf_ = dalloc((size_t)maxc * panel_wbuf_stride() * sizeof(T));
    }
    LIIs_ = dalloc(nLII_ * sizeof(T));
    Lrrs_ = dalloc(nLrr_ * sizeof(T));
    plan_int_.packed = LIIs_;
    plan_int_.poff = LII_off_;
    plan_rr_.packed = Lrrs_;
    plan_rr_.poff = Lrr_off_;
    slots_ = dalloc(nslot_ * sizeof(T));
    F_ = dalloc(nF_ * sizeof(T));
    Z_ = dalloc(nZ_ * sizeof(T));
    fac_ = dalloc(nfac_ * sizeof(T));
    inv_ = dalloc(nfac_ * sizeof(T));
    dmat_ = dalloc(nslot_ * sizeof(T));
    dmatT_ = dalloc(nslot_ * sizeof(T));
    Srr_ = feti ? dalloc(nSrr_ * sizeof(T)) : nullptr;
    xI_ = dalloc(nxI_ * sizeof(T));
    xr_ = dalloc(nxr_ * sizeof(T));
    xr2_ = dalloc(nxr_ * sizeof(T));
    Svv_ = (double*)dalloc((size_t)nsub * SVV_STRIDE * sizeof(double));
    Sp_ = (double*)dalloc((size_t)nsub * SP_STRIDE * sizeof(double));
    cP_ = (double*)dalloc((size_t)nsub * MAXP * sizeof(double));
    mu_ = (double*)dalloc((size_t)nsub * MAXC * sizeof(double));
    const int np = topo.nprimal;
    cb_ = (double*)dalloc((size_t)np * sizeof(double));
    {
        const std::string e = coarse_.alloc(ctx_alloc, &allocs_, stream_);
        if (!e.empty()) {
            set_error(e);
            return BDM_E_OOM;
        }
    }
    ybuf_ = (double*)dalloc(nyb_ * sizeof(double));
    info_sub_ = (int*)dalloc(nsub * sizeof(int));
    info_obj_ = (int*)dalloc((size_t)od_.nobj * sizeof(int));
    info_c_ = (int*)dalloc(sizeof(int));
    // the second workspace only with more than one chunk and 16 GB to spare
    // after it (Krylov vectors and the network come later)
    if (setup_overlap_ && chunks_.size() > 1) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && fr > (size_t)nKwork_ * sizeof(T) + ((size_t)16 << 30))
            K2_ = dalloc(nKwork_ * sizeof(T));
    }
    if (!K_ || !Wbuf_ || !LIIs_ || !Lrrs_ || !slots_ || !inv_ || !dmat_ || !dmatT_ || !F_ || !Z_ || !fac_ || (feti && !Srr_) || !xI_ || !xr_ ||
        !xr2_ || !Svv_ || !Sp_ || !cP_ || !mu_ || !cb_ || !ybuf_ || !info_sub_ || !info_obj_ || !info_c_) {
        set_error("device allocation failed (local factors)");
        return BDM_E_OOM;
    }
    return 0;
}

int Context::set_state(const double* v, const double* ue, const double* w, double t, bool dev) {
    const size_t vb = (size_t)N * sizeof(double);
    const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (v) HIPOK(hipMemcpyAsync(v_, v, vb, k, stream_)); else HIPOK(hipMemsetAsync(v_, 0, vb, stream_));
    if (ue) HIPOK(hipMemcpyAsync(ue_, ue, vb, k, stream_)); else HIPOK(hipMemsetAsync(ue_, 0, vb, stream_));
    if (w) HIPOK(hipMemcpyAsync(w_, w, vb, k, stream_)); else HIPOK(hipMemsetAsync(w_, 0, vb, stream_));
    launch_sub_mean(stream_, N, ue_, part_, tick_, scal_);
    HIPOK(hipMemcpyAsync(vn_, v_, vb, hipMemcpyDeviceToDevice, stream_));
    t_ = t;
    nstep_ = 0;
    have_prev_ = false;
    return sync();
}

int Context::get_state(double* v, double* ue, double* w, double* t, bool dev) {
    const size_t vb = (size_t)N * sizeof(double);
    const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (v) HIPOK(hipMemcpyAsync(v, v_, vb, k, stream_));
    if (ue) HIPOK(hipMemcpyAsync(ue, ue_, vb, k, stream_));
    if (w) HIPOK(hipMemcpyAsync(w, w_, vb, k, stream_));
    if (t) *t = t_;
    return sync();
}

int Context::set_stimulus(const double* Is, int on, int off, bool dev) {
    const size_t vb = (size_t)N * sizeof(double);
    if (Is) {
        HIPOK(hipMemcpyAsync(Is_, Is, vb, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, stream_));
        have_stim_ = true;
    } else {
        HIPOK(hipMemsetAsync(Is_, 0, vb, stream_));
        have_stim_ = false;
    }
    stim_on_ = on;
    stim_off_ = off;
    return sync();
}

int Context::ionic_update() {
    launch_ionic_update(stream_, fp, v_, w_);
    return sync();
}

int Context::residual(const double* v, const double* ue, double* Rv, double* Re) {
    HIPOK(hipMemcpyAsync(vn_, v_, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, stream_));
    const double stim = (have_stim_ && nstep_ >= stim_on_ && nstep_ < stim_off_) ? 1.0 : 0.0;
    launch_residual(stream_, fp, st_, v, ue, vn_, w_, Is_, stim, Rv, Re);
    return sync();
}

int Context::jacobian_apply(const double* x, double* y) {
    if (!linearized_) {
        set_error("bdm_jacobian_apply before bdm_linearize");
        return BDM_E_STATE;
    }
    launch_jac_apply(stream_, fp, st_, dg_, x, y);
    return sync();
}

// Launch sizes of an elimination plan for rank-k variant `variant`: tiles
// per matrix and panel row blocks, max over the subdomains.
void Context::build_plan(ElimPlan& pl, bool interior, int variant) {
    const int wp = interior_panel_width();
    int maxne = 0;
    for (const auto& sb : topo.subs) maxne = std::max(maxne, interior ? sb.nI : sb.nr);
    pl.variant = variant;
    pl.trail.assign((maxne + wp - 1) / wp, 0);
    pl.rows.assign(pl.trail.size(), 0);
    pl.schur = 0;
    for (const auto& sb : topo.subs) {
        const int e = interior ? sb.nI : sb.nr, m = interior ? sb.n() : sb.nr, c = interior ? sb.nIc : 0;
        for (size_t q = 0; q < pl.trail.size(); ++q) {
            pl.trail[q] = std::max(pl.trail[q], syrk_tiles(false, (int)q * wp, e, m, variant, c));
            pl.rows[q] = std::max(pl.rows[q], panel_rowblocks((int)q * wp, e, m, c));
        }
        if (interior) pl.schur = std::max(pl.schur, syrk_tiles(true, 0, e, m, variant));
    }
}

// Median of `reps` timed launches of fn on the context stream (ms), after
// one untimed launch.
static double time_launches(hipStream_t s, int reps, const std::function<void()>& fn) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1.0;
    if (hipEventCreate(&b) != hipSuccess) {
        hipEventDestroy(a);
        return -1.0;
    }
    fn();
    std::vector<double> t;
    for (int r = 0; r < reps; ++r) {
        hipEventRecord(a, s);
        fn();
        hipEventRecord(b, s);
        float ms = -1.f;
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = -1.f;
        t.push_back(ms);
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    std::sort(t.begin(), t.end());
    return (hipGetLastError() == hipSuccess) ? t[t.size() / 2] : -1.0;
}

// Stencil tile shape for this mesh: the fused Jacobian apply timed with
// every shape (it only reads its inputs, so the timing is repeatable).
int Context::tune_stencil() {
    char cls[96];
    std::snprintf(cls, sizeof cls, "mesh %dx%dx%d", fp.nx, fp.ny, fp.nz);
    launch_fill(stream_, 2 * N, 0.0, kp_);
    launch_fill(stream_, N, 0.0, dg_);
    fp.stencil_variant = tuner_.pick("stencil", cls, stencil_variants(), [&](int v) {
        fp.stencil_variant = v;
        return time_launches(stream_, 5, [&] { launch_jac_apply(stream_, fp, st_, dg_, kp_, kq_); });
    });
    HIPOK(hipStreamSynchronize(stream_));
    HIPOK(hipGetLastError());
    return 0;
}

// Rank-k variants of the interior and r-block elimination plans, timed on the
// first chunk's workspace before its first assembly (the trailing update after
// the first panel and, for the interior plan, the Schur update; the workspace
// is cleared again by the assembly).
template <typename T>
int Context::tune_syrk() {
    const int s0 = chunks_[0].first, cnt = chunks_[0].second - chunks_[0].first;
    T* K = (T*)K_;
    int maxnI = 0, maxn = 0, maxnr = 0;
    for (int q = s0; q < s0 + cnt; ++q) {
        maxnI = std::max(maxnI, topo.subs[q].nI);
        maxn = std::max(maxn, topo.subs[q].n());
        maxnr = std::max(maxnr, topo.subs[q].nr);
    }
    launch_fill_t<T>(stream_, nKwork_, (T)1e-3, K);
    for (int interior = 1; interior >= 0; --interior) {
        ElimPlan& pl = interior ? plan_int_ : plan_rr_;
        char cls[128];
        std::snprintf(cls, sizeof cls, "%s %s nsub=%d ne<=%d n<=%d", prec_ ? "f32" : "f64",
                      interior ? "interior" : "rblock", cnt, interior ? maxnI : maxnr, interior ? maxn : maxnr);
        const int v = tuner_.pick("syrk", cls, syrk_variants(), [&](int var) {
            ElimPlan tp = pl;
            tp.off = pl.off;
            tp.ne = pl.ne;
            tp.n = pl.n;
            build_plan(tp, interior != 0, var);
            if (tp.trail.empty() || (tp.trail[0] <= 0 && tp.schur <= 0)) return -1.0;
            return time_launches(stream_, 3, [&] {
                if (tp.trail[0] > 0)
                    launch_syrk_update<T>(stream_, cnt, K, tp.off + s0, ld_ + s0, tp.ne + s0, tp.n + s0, false, 0,
                                          tp.trail[0], var, tp.nIc ? tp.nIc + s0 : nullptr);
                if (tp.schur > 0)
                    launch_syrk_update<T>(stream_, cnt, K, tp.off + s0, ld_ + s0, tp.ne + s0, tp.n + s0, true, 0,
                                          tp.schur, var, tp.nIc ? tp.nIc + s0 : nullptr);
            });
        });
        const int64_t* off = pl.off;
        const int *ne = pl.ne, *n = pl.n;
        build_plan(pl, interior != 0, v);
        pl.off = off;
        pl.ne = ne;
        pl.n = n;
    }
    HIPOK(hipStreamSynchronize(stream_));
    HIPOK(hipGetLastError());
    syrk_tuned_ = true;
    return save_tuning();
}

int Context::side_stream_init() {
    if (side_stream_) return 0;
    HIPOK(hipStreamCreateWithFlags(&side_stream_, hipStreamNonBlocking));
    for (hipEvent_t* e : {&ev_fork_, &ev_join_, &ev_free_, &ev_ready_})
        HIPOK(hipEventCreateWithFlags(e, hipEventDisableTiming));
    return 0;
}

int Context::save_tuning() {
    if (tune_path_.empty() || !tuner_.dirty) return 0;
    const std::string e = tuner_.save(tune_path_);
    if (!e.empty()) {
        set_error(e);
        return BDM_E_ARG;
    }
    tuner_.dirty = false;
    return 0;
}

int Context::linearize(const double* v, const double* w) {
    const size_t vb = (size_t)N * sizeof(double);
    HIPOK(hipMemcpyAsync(vlin_, v, vb, hipMemcpyDeviceToDevice, stream_));
    HIPOK(hipMemcpyAsync(wlin_, w, vb, hipMemcpyDeviceToDevice, stream_));
    int rc = prec_ ? linearize_t<float>() : linearize_t<double>();
    if (rc == 0) linearized_ = true;
    return rc;
}

// Right-looking blocked Cholesky of the local matrices of one chunk in
// panels (see ElimPlan).  With timing, tm[0] and tm[1] accumulate the
// durations (ms) of the panel kernels and of the rank-k update kernel, tm[2]
// and tm[3] count their launches.
template <typename T>
int Context::eliminate(T* K, int s0, int cnt, const ElimPlan& pl, double* tm) {
    const int w = interior_panel_width();
    hipEvent_t ev[3];
    if (tm)
        for (auto& e : ev) HIPOK(hipEventCreate(&e));
    auto mark = [&](int q) -> int {
        if (tm) HIPOK(hipEventRecord(ev[q], stream_));
        return 0;
    };
    auto lap = [&](int a, int b, double& acc) -> int {
        if (!tm) return 0;
        HIPOK(hipEventSynchronize(ev[b]));
        float ms = 0.f;
        HIPOK(hipEventElapsedTime(&ms, ev[a], ev[b]));
        acc += ms;
        return 0;
    };
    for (int q = 0; q < (int)pl.trail.size(); ++q) {
        const int J = q * w;
        mark(0);
        launch_interior_panel<T>(stream_, cnt, K, pl.off + s0, ld_ + s0, pl.ne + s0, pl.n + s0, J, (T*)Wbuf_,
                                 pl.rows[q], info_sub_ + s0, (T*)pl.packed, pl.poff ? pl.poff + s0 : nullptr,
                                 pl.nIc ? pl.nIc + s0 : nullptr);
        mark(1);
        launch_syrk_update<T>(stream_, cnt, K, pl.off + s0, ld_ + s0, pl.ne + s0, pl.n + s0, false, J, pl.trail[q],
                              pl.variant, pl.nIc ? pl.nIc + s0 : nullptr);
        mark(2);
        if (tm) {
            lap(0, 1, tm[0]);
            lap(1, 2, tm[1]);
            tm[2] += pl.rows[q] > 0 ? 2 : 1;
            tm[3] += pl.trail[q] > 0 ? 1 : 0;
        }
    }
    if (pl.schur > 0) {
        mark(0);
        launch_syrk_update<T>(stream_, cnt, K, pl.off + s0, ld_ + s0, pl.ne + s0, pl.n + s0, true, 0, pl.schur,
                              pl.variant, pl.nIc ? pl.nIc + s0 : nullptr);
        mark(1);
        if (tm) {
            lap(0, 1, tm[1]);
            tm[3] += 1;
        }
    }
    if (tm)
        for (auto& e : ev) hipEventDestroy(e);
    return 0;
}

template <typename T>
int Context::linearize_t() {
    if (!syrk_tuned_) {
        const int trc = tune_syrk<T>();
        if (trc) return trc;
    }
    const int nsub = (int)topo.subs.size();
    const int np = topo.nprimal;
    HIPOK(hipMemsetAsync(bad_, 0, sizeof(int), stream_));
    launch_reaction_diag(stream_, fp, vlin_, wlin_, dg_, bad_);
    T* K = (T*)K_;
    HIPOK(hipMemsetAsync(info_sub_, 0, nsub * sizeof(int), stream_));
    HIPOK(hipMemsetAsync(info_obj_, 0, od_.nobj * sizeof(int), stream_));
    HIPOK(hipMemsetAsync(info_c_, 0, sizeof(int), stream_));
    HIPOK(hipMemsetAsync(F_, 0, nF_ * sizeof(T), stream_));
    // With a second workspace, chunk c + 1 is cleared and assembled on the
    // side stream while chunk c is eliminated here: the side stream waits
    // until the chunk that last used that workspace (c - 1) is done, and
    // chunk c + 1 waits for its assembly.
    const int nch = (int)chunks_.size();
    const bool ovl = K2_ != nullptr && nch > 1;
    if (ovl) {
        if (const int rc = side_stream_init()) return rc;
    }
    T* Kbuf[2] = {K, ovl ? (T*)K2_ : K};
    auto prepare = [&](hipStream_t st, int c, T* Kc) {
        BatchDesc cd = bd_;
        cd.nsub = chunks_[c].second - chunks_[c].first;
        cd.sub0 = chunks_[c].first;
        launch_clear_lower<T>(st, cd, maxn_, Kc);
        launch_assemble<T>(st, cd, maxbox_, fp, ke_, vlin_, wlin_, Kc);
    };
    for (int c = 0; c < nch; ++c) {
        const int s0 = chunks_[c].first, cnt = chunks_[c].second - chunks_[c].first;
        BatchDesc cd = bd_;
        cd.nsub = cnt;
        cd.sub0 = s0;
        T* Kc = Kbuf[c & 1];
        if (!ovl || c == 0) prepare(stream_, c, Kc);
        else HIPOK(hipStreamWaitEvent(stream_, ev_ready_, 0));
        if (ovl && c + 1 < nch) {
            HIPOK(hipEventRecord(ev_free_, stream_));
            HIPOK(hipStreamWaitEvent(side_stream_, ev_free_, 0));
            prepare(side_stream_, c + 1, Kbuf[(c + 1) & 1]);
            HIPOK(hipEventRecord(ev_ready_, side_stream_));
        }
        // interior elimination: L_II, L_GI and S_Gamma in the trailing block (Sec. 4.1)
        eliminate<T>(Kc, s0, cnt, plan_int_, nullptr);
        launch_extract<T>(stream_, cd, Kc, (T*)slots_, (T*)F_, Svv_, (T*)Srr_);
        // constrained Neumann factor L_rr of S_rr (the leading r-block of S_Gamma);
        // the panel kernels of both eliminations also write the factors into
        // their panel-packed storage
        eliminate<T>(Kc, s0, cnt, plan_rr_, nullptr);
    }
    // The deluxe factors need only the extracted blocks: they run on the side
    // stream while the coarse factorization (whose upper tree levels leave
    // most of the device idle) runs here; the two join before the status
    // read-back.
    if (const int rc = side_stream_init()) return rc;
    // The coarse basis algebra runs before the fork: alone it takes a third
    // of its time beside the deluxe kernels, which then overlap the coarse
    // factorization only.
    launch_trsm_fwd<T>(stream_, nsub, (const T*)Lrrs_, Lrr_off_, nr_, (T*)F_, bd_.F_off, nr_, kF_);
    launch_coarse_local<T>(stream_, bd_, (const T*)F_, Svv_, (T*)Z_, Sp_, info_sub_);
    HIPOK(hipEventRecord(ev_fork_, stream_));
    HIPOK(hipStreamWaitEvent(side_stream_, ev_fork_, 0));
    if (opts.scaling == BDM_SCALING_RHO) {
        launch_rho_fill<T>(side_stream_, od_, rho_w_, (T*)dmat_, (T*)dmatT_);
    } else {
        // faces and edges separately: each launch reserves LDS for its own largest object
        launch_deluxe_setup<T>(side_stream_, od_, 0, nface_obj_, maxface_n_, (const T*)slots_, (T*)fac_,
                               (T*)dmat_, info_obj_);
        launch_deluxe_setup<T>(side_stream_, od_, nface_obj_, od_.nobj - nface_obj_, maxedge_n_,
                               (const T*)slots_, (T*)fac_, (T*)dmat_, info_obj_);
        launch_deluxe_transpose<T>(side_stream_, od_, (const T*)dmat_, (T*)dmatT_);
    }
    HIPOK(hipEventRecord(ev_join_, side_stream_));
    coarse_.factor(stream_, color_list_, color_ptr_, nP_, Sp_, SP_STRIDE);
    HIPOK(hipStreamWaitEvent(stream_, ev_join_, 0));
    int hb = 0, hc = 0;
    std::vector<int> hs(nsub), ho(od_.nobj);
    HIPOK(hipMemcpyAsync(&hb, bad_, sizeof(int), hipMemcpyDeviceToHost, stream_));
    HIPOK(hipMemcpyAsync(hs.data(), info_sub_, nsub * sizeof(int), hipMemcpyDeviceToHost, stream_));
    HIPOK(hipMemcpyAsync(ho.data(), info_obj_, od_.nobj * sizeof(int), hipMemcpyDeviceToHost, stream_));
    HIPOK(hipMemcpyAsync(&hc, coarse_.info, sizeof(int), hipMemcpyDeviceToHost, stream_));
    HIPOK(hipStreamSynchronize(stream_));
    HIPOK(hipGetLastError());
    if (hb) {
        set_error("reaction diagonal not positive: the coercivity hypothesis chi*Cm + tau dI/dv > 0 fails");
        return BDM_E_COERCIVITY;
    }
    for (int q = 0; q < nsub; ++q)
        if (hs[q]) {
            set_error("local factorisation failed in subdomain " + std::to_string(q));
            return BDM_E_NOT_SPD;
        }
    for (int q = 0; q < od_.nobj; ++q)
        if (ho[q]) {
            set_error("deluxe factorisation failed for object " + std::to_string(q));
            return BDM_E_NOT_SPD;
        }
    if (hc) {
        set_error("coarse factorisation failed");
        return BDM_E_NOT_SPD;
    }
    return 0;
}

// out(interior dofs) = K_II^{-1} (r - q)_I per subdomain (q may be null).
template <typename T>
void Context::dirichlet(const double* r, const double* q, double* out) {
    T* xI = (T*)xI_;
    launch_gather_I<T>(stream_, nInodes_, Ilist_, N, r, q, xI);
    if (fused_dirichlet_) {
        launch_trsv_fb<T>(stream_, bd_.nsub, (const T*)LIIs_, LII_off_, nI_, xI, xI_off_, maxnI_, qI_);
    } else {
        launch_trsv<T>(stream_, bd_.nsub, false, (const T*)LIIs_, LII_off_, nI_, xI, xI_off_, maxnI_, qI_);
        launch_trsv<T>(stream_, bd_.nsub, true, (const T*)LIIs_, LII_off_, nI_, xI, xI_off_, maxnI_, qI_);
    }
    launch_scatter_I<T>(stream_, nInodes_, Ilist_, N, xI, out);
}

// g = r - sum_j R_j^T K_GI K_II^{-1} r_I (interface rows of g are used)
template <typename T>
void Context::condense(const double* r, double* g) {
    launch_fill(stream_, 2 * N, 0.0, t1_);
    dirichlet<T>(r, nullptr, t1_);
    launch_res_minus_jac(stream_, fp, st_, dg_, t1_, r, g);
}

// S~^{-1} on local r-residuals in xr (Sec. 4.4): forward Neumann solve,
// coarse right-hand side (vertex residuals from gvert), coarse solve, and one
// backward solve for the Neumann correction plus the coarse prolongation.
template <typename T>
void Context::stilde_inv(T* xr, const double* gvert, double* uc) {
    launch_trsv<T>(stream_, bd_.nsub, false, (const T*)Lrrs_, Lrr_off_, nr_, xr, xr_off_, maxnr_, qr_);
    launch_coarse_rhs_local<T>(stream_, sv_, xr, (const T*)Z_, cP_, mu_);
    launch_coarse_rhs_gather(stream_, cd_, N, gvert, cP_, uc);
    launch_coarse_project(stream_, cd_.np, pin_, uc);
    coarse_.solve(stream_, uc);
    launch_neumann_rhs<T>(stream_, sv_, (const T*)F_, (const T*)Z_, mu_, uc, xr, 1);
    launch_trsv<T>(stream_, bd_.nsub, true, (const T*)Lrrs_, Lrr_off_, nr_, xr, xr_off_, maxnr_, qr_);
}

// zbuf holds interface values (zero interior); fill the interior by the
// discrete harmonic extension plus the interior correction:
// z_I = K_II^{-1} (r_I - K_IG z_G).
template <typename T>
void Context::interior_extend(const double* r, double* zbuf) {
    launch_jac_apply(stream_, fp, st_, dg_, zbuf, t1_);
    dirichlet<T>(r, t1_, zbuf);
}

int Context::bddc_apply(const double* r, double* z) {
    if (!linearized_) {
        set_error("bdm_bddc_apply before bdm_linearize");
        return BDM_E_STATE;
    }
    int rc = prec_ ? bddc_apply_t<float>(r, z) : bddc_apply_t<double>(r, z);
    if (rc) return rc;
    return sync();
}

// interior_free: r vanishes on the subdomain interiors, so the condensation
// r_G - K_GI K_II^{-1} r_I leaves r unchanged and is skipped.
template <typename T>
int Context::bddc_apply_t(const double* r, double* z, bool interior_free) {
    const double* g = r;
    if (!interior_free) {
        condense<T>(r, t2_);
        g = t2_;
    }
    launch_deluxe_res<T>(stream_, od_, N, g, (const T*)dmat_, (T*)xr_, xr_off_);
    stilde_inv<T>((T*)xr_, g, cb_);
    launch_fill(stream_, 2 * N, 0.0, t3_);
    launch_deluxe_val<T>(stream_, od_, N, (const T*)dmatT_, (const T*)xr_, xr_off_, t3_);
    launch_vertex_val(stream_, cd_.nverts, cd_.vnode, N, cb_, t3_);
    interior_extend<T>(r, t3_);
    HIPOK(hipMemcpyAsync(z, t3_, 2 * N * sizeof(double), hipMemcpyDeviceToDevice, stream_));
    return 0;
}

int Context::fetidp_apply(int op, const double* in, double* out) {
    if (!linearized_) {
        set_error("bdm_fetidp_apply before bdm_linearize");
        return BDM_E_STATE;
    }
    if (opts.solver != BDM_SOLVER_FETIDP) {
        set_error("context was created without FETI-DP workspace (opts.solver)");
        return BDM_E_STATE;
    }
    int rc = prec_ ? fetidp_apply_t<float>(op, in, out) : fetidp_apply_t<double>(op, in, out);
    if (rc) return rc;
    return sync();
}

template <typename T>
int Context::fetidp_apply_t(int op, const double* in, double* out) {
    T* xr = (T*)xr_;
    T* xr2 = (T*)xr2_;
    switch (op) {
        case BDM_FETI_F:
            launch_feti_BT<T>(stream_, od_, fd_, in, xr, xr_off_);
            stilde_inv<T>(xr, gzero_, cb_);
            launch_feti_B<T>(stream_, od_, fd_, xr, xr_off_, out);
            return 0;
        case BDM_FETI_PRECOND:
            launch_feti_BDT<T>(stream_, od_, fd_, in, (const T*)dmat_, xr, xr_off_);
            launch_schur_mv<T>(stream_, sv_, (const T*)Srr_, Srr_off_, xr, xr2);
            launch_feti_BD<T>(stream_, od_, fd_, xr2, xr_off_, (const T*)dmat_, out);
            return 0;
        case BDM_FETI_RHS:
            condense<T>(in, t2_);
            launch_split_res<T>(stream_, od_, N, t2_, xr, xr_off_);
            stilde_inv<T>(xr, t2_, cb_);
            launch_feti_B<T>(stream_, od_, fd_, xr, xr_off_, out);
            return 0;
        case BDM_FETI_RECOVER: {
            condense<T>(in, t2_);
            launch_split_res<T>(stream_, od_, N, t2_, xr, xr_off_);
            launch_feti_BT<T>(stream_, od_, fd_, in + 2 * N, xr2, xr_off_);
            hipLaunchKernelGGL(k_sub_t<T>, dim3(nb(nxr_, 256)), dim3(256), 0, stream_, nxr_, (const T*)xr2, xr);
            stilde_inv<T>(xr, t2_, cb_);
            launch_fill(stream_, 2 * N, 0.0, t3_);
            launch_take_first<T>(stream_, od_, N, xr, xr_off_, t3_);
            launch_vertex_val(stream_, cd_.nverts, cd_.vnode, N, cb_, t3_);
            interior_extend<T>(in, t3_);
            HIPOK(hipMemcpyAsync(out, t3_, 2 * N * sizeof(double), hipMemcpyDeviceToDevice, stream_));
            return 0;
        }
        default:
            set_error("unknown FETI-DP operator");
            return BDM_E_ARG;
    }
}

// PCG (zero initial guess, unpreconditioned residual norm test, Polak-Ribiere
// beta; Sec. 4.1 and the Sec. 6 tolerances), on the full Jacobian with BDDC
// or on the FETI-DP multiplier system.  One iteration is two halves of
// device work: the operator half (q = A p, p.q, the fused x / r update with
// ||r||^2 and the stopping test) and the preconditioner half (z = M r, the
// fused z.r / z.q pass with beta, p = z + beta p).  The scalars alpha, beta,
// the dots and the state (running, converged, diverged, iteration limit)
// live in device slots; the host reads back the state and iteration count
// (16 bytes) once per iteration.  With opts.krylov_graph the two halves are
// captured once per operator and size, on a private non-blocking stream, as
// two HIP graphs and replayed (no memset nodes and no host synchronisation
// inside); the kernels, their order and the arithmetic are the same, so the
// iterates are bitwise equal.
int Context::pcg(int n, const double* b, double* x, bool feti, KrylovOut& out, bool reduced, double rref) {
    out = KrylovOut();
    const int maxit = opts.krylov_maxit;
    if (maxit > kry_hcap_) {
        set_error("krylov_maxit exceeds the Krylov iteration history");
        return BDM_E_ARG;
    }
    auto A = [&](const double* in, double* o) -> int {
        if (feti) return prec_ ? fetidp_apply_t<float>(BDM_FETI_F, in, o) : fetidp_apply_t<double>(BDM_FETI_F, in, o);
        launch_jac_apply(stream_, fp, st_, dg_, in, o);
        return 0;
    };
    auto M = [&](const double* in, double* o) -> int {
        if (feti)
            return prec_ ? fetidp_apply_t<float>(BDM_FETI_PRECOND, in, o)
                         : fetidp_apply_t<double>(BDM_FETI_PRECOND, in, o);
        return prec_ ? bddc_apply_t<float>(in, o, reduced) : bddc_apply_t<double>(in, o, reduced);
    };
    auto op_half = [&]() -> int {
        const int rc = A(kp_, kq_);
        if (rc) return rc;
        launch_dot(stream_, n, kp_, kq_, part_, tick_, kry_sc_ + PCG_PQ);
        launch_pcg_update(stream_, n, kry_sc_, kp_, kq_, x, kr_, part_, tick_, kry_hist_, kry_ah_, maxit);
        return 0;
    };
    auto prec_half = [&]() -> int {
        const int rc = M(kr_, kz_);
        if (rc) return rc;
        launch_pcg_beta(stream_, n, kry_sc_, kz_, kr_, kq_, part_, tick_, kry_bh_);
        launch_scale_add_dev(stream_, n, kz_, kry_sc_ + PCG_BETA, kp_);
        return 0;
    };
    // set-up, eager
    launch_fill(stream_, n, 0.0, x);
    launch_copy_kernel(stream_, n, b, kr_);
    const double r0 = std::sqrt(dot(n, kr_, kr_));
    if (hip_err_) return BDM_E_HIP;
    const double ref = rref > 0.0 ? rref : r0;
    out.hist.push_back(r0);
    if (r0 == 0.0) return 0;
    int rc = M(kr_, kz_);
    if (rc) return rc;
    launch_copy_kernel(stream_, n, kz_, kp_);
    launch_dot(stream_, n, kr_, kz_, part_, tick_, kry_sc_ + PCG_RZ);
    {
        double init[PCG_NSLOT] = {0};
        init[PCG_STATE] = PCG_RUNNING;
        init[PCG_IT] = 0;
        init[PCG_TOL] = opts.krylov_rtol * ref;
        init[PCG_DTOL] = opts.krylov_dtol * ref;
        // keep PCG_RZ (computed on the device above): copy the other slots only
        HIPOK(hipMemcpyAsync(kry_sc_ + PCG_PQ, init + PCG_PQ, (PCG_NSLOT - PCG_PQ) * sizeof(double),
                             hipMemcpyHostToDevice, stream_));
        HIPOK(hipStreamSynchronize(stream_));   // init lives on this host stack
    }
    const bool graph = opts.krylov_graph != 0;
    if (graph) {
        // capture both halves once per (operator, size)
        const int key = (feti ? 1 : 0) + (reduced ? 2 : 0) + 4 * n;
        if (!kry_exec_[0] || !kry_exec_[1] || kry_key_ != key) {
            for (auto& g : kry_exec_)
                if (g) {
                    hipGraphExecDestroy(g);
                    g = nullptr;
                }
            kry_key_ = -1;
            if (!kry_stream_) HIPOK(hipStreamCreateWithFlags(&kry_stream_, hipStreamNonBlocking));
            HIPOK(hipStreamSynchronize(stream_));
            for (int half = 0; half < 2; ++half) {
                hipStream_t saved = stream_;
                stream_ = kry_stream_;
                HIPOK(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
                const int brc = half == 0 ? op_half() : prec_half();
                hipGraph_t g = nullptr;
                const hipError_t ce = hipStreamEndCapture(stream_, &g);
                stream_ = saved;
                if (brc) {
                    if (g) hipGraphDestroy(g);
                    return brc;
                }
                HIPOK(ce);
                const hipError_t ie = hipGraphInstantiate(&kry_exec_[half], g, nullptr, nullptr, 0);
                hipGraphDestroy(g);
                HIPOK(ie);
            }
            kry_key_ = key;
            kry_x_ = x;
        }
        // the operator half writes x: its pointer is part of the captured graph
        if (x != kry_x_) {
            set_error("internal error: graph PCG called with a different solution vector");
            return BDM_E_STATE;
        }
    }
    double st[2] = {PCG_RUNNING, 0.0};
    for (int it = 0; it < maxit; ++it) {
        if (graph) HIPOK(hipGraphLaunch(kry_exec_[0], stream_));
        else if ((rc = op_half())) return rc;
        HIPOK(hipMemcpyAsync(st, kry_sc_ + PCG_STATE, 2 * sizeof(double), hipMemcpyDeviceToHost, stream_));
        HIPOK(hipStreamSynchronize(stream_));
        if (st[0] != PCG_RUNNING) break;
        if (graph) HIPOK(hipGraphLaunch(kry_exec_[1], stream_));
        else if ((rc = prec_half())) return rc;
    }
    const int its = (int)st[1];
    out.its = its;
    out.status = (st[0] == PCG_CONVERGED) ? 0 : (st[0] == PCG_DIVERGED ? 2 : 1);
    std::vector<double> h(its + 1), a(its), bb(std::max(its - 1, 0));
    HIPOK(hipMemcpyAsync(h.data(), kry_hist_, (its + 1) * sizeof(double), hipMemcpyDeviceToHost, stream_));
    if (its) HIPOK(hipMemcpyAsync(a.data(), kry_ah_, its * sizeof(double), hipMemcpyDeviceToHost, stream_));
    if (its > 1) HIPOK(hipMemcpyAsync(bb.data(), kry_bh_, (its - 1) * sizeof(double), hipMemcpyDeviceToHost, stream_));
    HIPOK(hipStreamSynchronize(stream_));
    h[0] = r0;
    out.hist = h;
    out.alpha = a;
    out.beta = bb;
    out.cond = lanczos_cond(out.alpha, out.beta);
    return 0;
}

int Context::krylov(int n, const double* b, double* x, bool feti, KrylovOut& out, bool reduced, double rref) {
    return pcg(n, b, x, feti, out, reduced, rref);
}

// J s = b with the configured preconditioner.
int Context::newton_solve(const double* b, double* s, KrylovOut& out) {
    // project the u_e block of b onto the range (zero sum)
    HIPOK(hipMemcpyAsync(Rt_, b, 2 * N * sizeof(double), hipMemcpyDeviceToDevice, stream_));
    launch_sub_mean(stream_, N, Rt_ + N, part_, tick_, scal_);
    if (opts.solver != BDM_SOLVER_FETIDP) {
        if (!opts.krylov_reduced) return krylov((int)(2 * N), Rt_, s, false, out);
        // s0 = interior solves of b, zero on the interface (Sec. 4.1); the
        // residual b - J s0 vanishes on every subdomain interior, and so do
        // all later PCG residuals, since each preconditioned direction ends
        // with the interior correction.  PCG then solves J s' = b - J s0 and
        // s = s0 + s'.  The stopping test is relative to ||b||, so the final
        // residual b - J s meets the same bound as the unreduced solve.
        // kx_ is unused by BDDC; pcg copies its right-hand side (kq_ here)
        // before it first writes kq_.
        const double bn = std::sqrt(dot(2 * N, Rt_, Rt_));
        launch_fill(stream_, 2 * N, 0.0, kx_);
        if (prec_) dirichlet<float>(Rt_, nullptr, kx_);
        else dirichlet<double>(Rt_, nullptr, kx_);
        launch_res_minus_jac(stream_, fp, st_, dg_, kx_, Rt_, kq_);
        const int rc = krylov((int)(2 * N), kq_, s, false, out, true, bn);
        if (rc) return rc;
        launch_axpy(stream_, 2 * N, 1.0, kx_, s);
        return 0;
    }
    // FETI-DP: d = B S~^{-1} f~, PCG on F lambda = d, then recovery.  d
    // (n_lambda values, which exceed 2N when the subdomains are small) stays
    // in kq_: pcg copies its right-hand side before it first writes kq_.
    int rc = prec_ ? fetidp_apply_t<float>(BDM_FETI_RHS, Rt_, kq_) : fetidp_apply_t<double>(BDM_FETI_RHS, Rt_, kq_);
    if (rc) return rc;
    rc = krylov((int)nlam_, kq_, kx_, true, out);
    if (rc) return rc;
    // recover: input [b ; lambda]
    HIPOK(hipMemcpyAsync(kq_, Rt_, 2 * N * sizeof(double), hipMemcpyDeviceToDevice, stream_));
    HIPOK(hipMemcpyAsync(kq_ + 2 * N, kx_, nlam_ * sizeof(double), hipMemcpyDeviceToDevice, stream_));
    rc = prec_ ? fetidp_apply_t<float>(BDM_FETI_RECOVER, kq_, s) : fetidp_apply_t<double>(BDM_FETI_RECOVER, kq_, s);
    return rc;
}

int Context::profile_kernel(int kernel, int reps, double* avg_ms, double* work) {
    if (!linearized_) {
        set_error("bdm_profile_kernel before bdm_linearize");
        return BDM_E_STATE;
    }
    if (reps < 1 || kernel < 0 || kernel > BDM_KERNEL_TRSV_DIRICHLET_T) {
        set_error("bdm_profile_kernel: bad kernel id or reps");
        return BDM_E_ARG;
    }
    return prec_ ? profile_t<float>(kernel, reps, avg_ms, work) : profile_t<double>(kernel, reps, avg_ms, work);
}

template <typename T>
int Context::profile_t(int kernel, int reps, double* avg_ms, double* work) {
    hipEvent_t e0, e1;
    HIPOK(hipEventCreate(&e0));
    HIPOK(hipEventCreate(&e1));
    double total = 0.0, w = 0.0;
    const int nsub = (int)topo.subs.size();
    const int s0 = chunks_[0].first, cnt = chunks_[0].second - chunks_[0].first;
    BatchDesc cd = bd_;
    cd.nsub = cnt;
    cd.sub0 = s0;
    if (kernel == BDM_KERNEL_JACOBIAN) {
        // vectors: x (2), the reaction diagonal and y (2) per node; mapped
        // meshes add the 54 per-node coefficients
        w = (fp.stn ? 40.0 + 54.0 * 8.0 : 40.0) * (double)N;
    } else if (kernel == BDM_KERNEL_TRSV_DIRICHLET || kernel == BDM_KERNEL_TRSV_DIRICHLET_T) {
        for (const auto& sb : topo.subs) w += (0.5 * sb.nI * (sb.nI + 1.0) + 2.0 * sb.nI) * sizeof(T);
    } else {
        // interior elimination flops: the panel kernel (divisions and the
        // updates inside each panel) and the update kernel (trailing updates
        // right of each panel and the Schur update), 2 flops per updated
        // entry.  Entries of the interface rows [nI, n) in the core columns
        // [0, nIc) are zero and stay zero, so neither they nor the products
        // they enter count.
        const int wp = interior_panel_width();
        auto tri = [](double c0, double c1, double n) {     // sum over columns [c0, c1) of (n - c)
            const double m = c1 - c0;
            return m > 0 ? m * n - (c0 + c1 - 1) * m / 2.0 : 0.0;
        };
        for (int q = s0; q < s0 + cnt; ++q) {
            const double n = topo.subs[q].n(), nI = topo.subs[q].nI, nIc = topo.subs[q].nIc, nG = n - nI;
            double wpanel = 0, wupd = 0;
            for (int J = 0; J < nI; J += wp) {
                const double pe = std::min<double>(J + wp, nI);
                for (int j = J; j < pe; ++j) {
                    const double g = j >= nIc ? nG : 0.0;      // interface rows of column j
                    wpanel += (nI - j - 1) + g + 2.0 * (tri(j + 1, pe, nI) + g * (pe - j - 1));
                }
                const double kg = std::max(0.0, pe - std::max<double>(J, nIc));   // inner indices for them
                const double cols = std::max(0.0, nI - (J + wp));
                wupd += 2.0 * ((pe - J) * tri(J + wp, nI, nI) + kg * cols * nG);
            }
            wupd += (nI - nIc) * nG * (nG + 1.0);
            w += (kernel == BDM_KERNEL_POTRF_INTERIOR) ? wpanel : wupd;
        }
    }
    double launches = 1.0;
    for (int r = 0; r < reps; ++r) {
        if (kernel == BDM_KERNEL_JACOBIAN || kernel == BDM_KERNEL_TRSV_DIRICHLET ||
            kernel == BDM_KERNEL_TRSV_DIRICHLET_T) {
            HIPOK(hipEventRecord(e0, stream_));
            if (kernel == BDM_KERNEL_JACOBIAN)
                launch_jac_apply(stream_, fp, st_, dg_, kp_, kq_);
            else
                launch_trsv<T>(stream_, nsub, kernel == BDM_KERNEL_TRSV_DIRICHLET_T, (const T*)LIIs_, LII_off_, nI_,
                               (T*)xI_, xI_off_, maxnI_, qI_);
            HIPOK(hipEventRecord(e1, stream_));
            HIPOK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPOK(hipEventElapsedTime(&ms, e0, e1));
            total += ms;
        } else {
            launch_clear_lower<T>(stream_, cd, maxn_, (T*)K_);
            launch_assemble<T>(stream_, cd, maxbox_, fp, ke_, vlin_, wlin_, (T*)K_);
            double tm[4] = {0.0, 0.0, 0.0, 0.0};
            int rc = eliminate<T>((T*)K_, s0, cnt, plan_int_, tm);
            if (rc) return rc;
            const bool panel = kernel == BDM_KERNEL_POTRF_INTERIOR;
            total += panel ? tm[0] : tm[1];
            launches = std::max(1.0, panel ? tm[2] : tm[3]);
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *avg_ms = total / (reps * launches);
    *work = w / launches;
    return 0;
}


int Context::ensure_predictor() {
    if (pred_.ready) return 0;
    const std::string e = pred_.init(N, fp.nx1, fp.ny1, fp.nz + 1, ctx_alloc, &allocs_);
    if (!e.empty()) {
        set_error(e);
        return BDM_E_OOM;
    }
    return 0;
}

int Context::predictor_set(const float* params, const double* scales) {
    int rc = ensure_predictor();
    if (rc) return rc;
    for (int q = 0; q < kScales; ++q)
        if (!(scales[q] > 0)) {
            set_error("predictor scales must be positive");
            return BDM_E_ARG;
        }
    pred_.set(stream_, params, scales);
    HIPOK(hipGetLastError());
    return 0;
}

int Context::predictor_get(float* params, double* scales) {
    if (!pred_.has_weights) {
        set_error("predictor has no weights");
        return BDM_E_STATE;
    }
    pred_.get(stream_, params, scales);
    return 0;
}

int Context::predictor_guess(const double* vn, const double* uen, const double* vp, const double* uep, double* out) {
    if (!pred_.has_weights) {
        set_error("predictor has no weights");
        return BDM_E_STATE;
    }
    pred_.guess(stream_, vn, uen, vp, uep, out);
    return sync();
}

int Context::predictor_loss_grad(const double* sample, float* grad, double* loss) {
    if (!pred_.has_weights) {
        set_error("predictor has no weights");
        return BDM_E_STATE;
    }
    *loss = pred_.loss_grad(stream_, sample);
    HIPOK(hipMemcpyAsync(grad, pred_.grad, Predictor::n_params() * sizeof(float), hipMemcpyDeviceToHost, stream_));
    return sync();
}

int Context::predictor_train(const double* samples, int nsamples, const int* order, int nsteps, double lr,
                             double* losses) {
    if (!pred_.has_weights) {
        set_error("predictor has no weights");
        return BDM_E_STATE;
    }
    for (int t = 0; t < nsteps; ++t) {
        if (order[t] < 0 || order[t] >= nsamples) {
            set_error("training order index out of range");
            return BDM_E_ARG;
        }
        const double l = pred_.train_step(stream_, samples + (int64_t)order[t] * 6 * N, lr);
        if (losses) losses[t] = l;
    }
    HIPOK(hipGetLastError());
    return sync();
}

int Context::step(int nsteps, bdm_step_stats* st) {
    using clk = std::chrono::steady_clock;
    const size_t vb = (size_t)N * sizeof(double);
    if (opts.solver == BDM_SOLVER_FETIDP && prec_) {
        // the multiplier operator holds the local solves: with FP32 factors it
        // loses definiteness (negative Lanczos estimates, PCG breakdown)
        set_error("FETI-DP Newton solves need FP64 local factors (precision BDM_PREC_FP64)");
        return BDM_E_ARG;
    }
    for (int ks = 0; ks < nsteps; ++ks) {
        bdm_step_stats S{};
        S.bad_subdomain = -1;
        const auto t0 = clk::now();
        double tsetup = 0, tkry = 0;
        // Step 1: gating update from v^n (Sec. 3b)
        HIPOK(hipMemcpyAsync(vn_, v_, vb, hipMemcpyDeviceToDevice, stream_));
        launch_ionic_update(stream_, fp, v_, w_);
        const double stim = (have_stim_ && nstep_ >= stim_on_ && nstep_ < stim_off_) ? 1.0 : 0.0;
        // reference residual ||R(u^n)||
        launch_residual(stream_, fp, st_, v_, ue_, vn_, w_, Is_, stim, R_, R_ + N);
        hip_err_ = false;
        const double ref = std::sqrt(dot(2 * N, R_, R_));
        if (hip_err_) return BDM_E_HIP;
        S.res_ref = ref;
        // initial guess: u^n, extrapolation, or the better (smaller ||R||) of the
        // learned and the extrapolated guess
        S.guess_used = 0;
        S.guess_res_extrap = -1.0;
        S.guess_res_cnn = -1.0;
        double rn;
        if (opts.guess != BDM_GUESS_PREV && have_prev_) {
            hipLaunchKernelGGL(k_lin_comb, dim3(nb(N, 256)), dim3(256), 0, stream_, N, 2.0, v_, -1.0, vprev_, U_);
            hipLaunchKernelGGL(k_lin_comb, dim3(nb(N, 256)), dim3(256), 0, stream_, N, 2.0, ue_, -1.0, ueprev_, U_ + N);
            launch_residual(stream_, fp, st_, U_, U_ + N, vn_, w_, Is_, stim, R_, R_ + N);
            rn = std::sqrt(dot(2 * N, R_, R_));
            S.guess_used = 1;
            S.guess_res_extrap = rn;
            if (opts.guess == BDM_GUESS_CNN && pred_.has_weights) {
                pred_.guess(stream_, v_, ue_, vprev_, ueprev_, Rt_);
                launch_residual(stream_, fp, st_, Rt_, Rt_ + N, vn_, w_, Is_, stim, kq_, kq_ + N);
                const double rc = std::sqrt(dot(2 * N, kq_, kq_));
                S.guess_res_cnn = rc;
                if (rc < rn) {
                    HIPOK(hipMemcpyAsync(U_, Rt_, 2 * vb, hipMemcpyDeviceToDevice, stream_));
                    HIPOK(hipMemcpyAsync(R_, kq_, 2 * vb, hipMemcpyDeviceToDevice, stream_));
                    rn = rc;
                    S.guess_used = 2;
                }
            }
        } else {
            HIPOK(hipMemcpyAsync(U_, v_, vb, hipMemcpyDeviceToDevice, stream_));
            HIPOK(hipMemcpyAsync(U_ + N, ue_, vb, hipMemcpyDeviceToDevice, stream_));
            launch_residual(stream_, fp, st_, U_, U_ + N, vn_, w_, Is_, stim, R_, R_ + N);
            rn = std::sqrt(dot(2 * N, R_, R_));
        }
        S.res_hist[0] = rn;
        int it = 0;
        int status = 0;
        for (; it < opts.newton_maxit; ++it) {
            if (rn <= std::max(opts.newton_rtol * ref, opts.newton_atol)) break;
            if (it >= 32) break;
            const auto ts = clk::now();
            int rc = linearize(U_, w_);
            tsetup += std::chrono::duration<double, std::milli>(clk::now() - ts).count();
            if (rc) return rc;
            // s = J^{-1} (-R)
            launch_scale_add(stream_, 2 * N, gzero_, -1.0, R_);   // R <- -R
            KrylovOut ko;
            const auto tk = clk::now();
            rc = newton_solve(R_, S_, ko);
            tkry += std::chrono::duration<double, std::milli>(clk::now() - tk).count();
            if (rc) return rc;
            // error of this solve, recomputed in FP64 on the full system:
            // ||b - J s|| / ||b|| with b the projected right-hand side (Rt_)
            launch_res_minus_jac(stream_, fp, st_, dg_, S_, Rt_, t1_);
            const double bn = std::sqrt(dot(2 * N, Rt_, Rt_));
            S.krylov_true_res[it] = bn > 0 ? std::sqrt(dot(2 * N, t1_, t1_)) / bn : 0.0;
            launch_scale_add(stream_, 2 * N, gzero_, -1.0, R_);   // restore R
            S.krylov_its[it] = ko.its;
            S.cond[it] = ko.cond;
            if (ko.status == 2) {
                set_error("Krylov iteration diverged");
                status = BDM_E_KRYLOV_DIVERGED;
                break;
            }
            if (ko.status == 1) status = BDM_E_KRYLOV_MAXIT;
            // line search on f = ||R||^2 / 2 (Sec. 6: Armijo test, then
            // backtracking by the minimiser of a quadratic model after the
            // first failure and of a cubic model after later ones, each new
            // step kept in [0.1, 0.5] of the previous; a non-finite f is not
            // modelled but halves the step)
            const double f0 = 0.5 * rn * rn, g0 = -2.0 * f0, alpha = 1e-4;
            double lam = 1.0, lam_prev = 0.0, f_prev = 0.0, f = 0.0;
            bool accepted = false, modelled = false;
            for (int ls = 0; ls < 20; ++ls) {
                HIPOK(hipMemcpyAsync(Rt_, U_, 2 * vb, hipMemcpyDeviceToDevice, stream_));
                launch_axpy(stream_, 2 * N, lam, S_, Rt_);
                launch_residual(stream_, fp, st_, Rt_, Rt_ + N, vn_, w_, Is_, stim, kq_, kq_ + N);
                f = 0.5 * dot(2 * N, kq_, kq_);
                if (std::isfinite(f) && f <= f0 + alpha * lam * g0) {
                    accepted = true;
                    break;
                }
                if (!std::isfinite(f)) {
                    lam *= 0.5;
                    continue;
                }
                double lt;
                if (!modelled) {
                    lt = -g0 / (2.0 * (f - f0 - g0));
                    modelled = true;
                } else {
                    const double r1 = f - f0 - lam * g0, r2 = f_prev - f0 - lam_prev * g0;
                    const double a = (r1 / (lam * lam) - r2 / (lam_prev * lam_prev)) / (lam - lam_prev);
                    const double b = (-lam_prev * r1 / (lam * lam) + lam * r2 / (lam_prev * lam_prev)) / (lam - lam_prev);
                    if (a == 0.0) lt = -g0 / (2.0 * b);
                    else lt = (-b + std::sqrt(std::max(b * b - 3.0 * a * g0, 0.0))) / (3.0 * a);
                }
                lam_prev = lam;
                f_prev = f;
                lam = std::min(std::max(lt, 0.1 * lam), 0.5 * lam);
            }
            S.step_length[it] = lam;
            if (hip_err_) return BDM_E_HIP;
            if (!accepted) {
                set_error("line search: no step along the Newton direction passed the Armijo test in 20 trials");
                status = BDM_E_LINESEARCH;
                ++it;
                break;
            }
            HIPOK(hipMemcpyAsync(U_, Rt_, 2 * vb, hipMemcpyDeviceToDevice, stream_));
            HIPOK(hipMemcpyAsync(R_, kq_, 2 * vb, hipMemcpyDeviceToDevice, stream_));
            launch_sub_mean(stream_, N, U_ + N, part_, tick_, scal_);
            rn = std::sqrt(2.0 * f);
            S.res_hist[it + 1] = rn;
        }
        S.newton_its = it;
        if (status == 0 && it >= opts.newton_maxit && rn > std::max(opts.newton_rtol * ref, opts.newton_atol)) {
            set_error("Newton iteration limit reached");
            status = BDM_E_NEWTON_MAXIT;
        }
        // history for extrapolation, then the new state
        HIPOK(hipMemcpyAsync(vprev_, v_, vb, hipMemcpyDeviceToDevice, stream_));
        HIPOK(hipMemcpyAsync(ueprev_, ue_, vb, hipMemcpyDeviceToDevice, stream_));
        have_prev_ = true;
        HIPOK(hipMemcpyAsync(v_, U_, vb, hipMemcpyDeviceToDevice, stream_));
        HIPOK(hipMemcpyAsync(ue_, U_ + N, vb, hipMemcpyDeviceToDevice, stream_));
        int rc = sync();
        if (rc) return rc;
        ++nstep_;
        t_ += opts.dt;
        S.t_setup_ms = tsetup;
        S.t_krylov_ms = tkry;
        S.t_step_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
        if (st) *st = S;
        if (status) return status;
    }
    return 0;
}

}  // namespace bdm
