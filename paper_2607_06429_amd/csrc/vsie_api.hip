// C ABI of libvsie.so: validation, device data, operator application and the
// GMRES solver with FP64 iterative refinement.  See include/vsie.h.
#include <algorithm>
#include <chrono>
#include <atomic>
#include <cmath>
#include <complex>
#include <functional>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include <rocblas/rocblas.h>

#include "vsie_internal.h"

namespace vsie {

thread_local std::string g_last_error;

void check_blas(rocblas_status st, const char *what) {
    if (st == rocblas_status_success) return;
    fail(st == rocblas_status_memory_error ? VSIE_E_NOMEM : VSIE_E_DEVICE,
         std::string(what) + ": " + rocblas_status_to_string(st));
}

void fail(vsie_status code, const std::string &msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    const vsie_status code = (e == hipErrorOutOfMemory) ? VSIE_E_NOMEM : VSIE_E_DEVICE;
    fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

// Epoch of every device address a captured operator graph may hold: bumped
// whenever a work buffer is reallocated or a problem's sources, tuning or
// assembled operators change.  A graph captured in an older epoch is never
// launched again.
std::atomic<uint64_t> g_graph_epoch{0};

// Grow-only device buffer.  During a call made with a caller workspace the
// buffer is a planned part of that workspace instead (ov_on): the call then
// never allocates, and asking for more than was planned is an error.
struct Scratch {
    void *p = nullptr;
    size_t bytes = 0;
    void *ov = nullptr;
    size_t ov_bytes = 0;
    bool ov_on = false;
    void *get(size_t b) {
        if (ov_on) {
            if (b > ov_bytes)
                fail(VSIE_E_WORKSPACE, "a work buffer needs " + std::to_string(b) + " bytes, its planned part of the "
                                       "workspace holds " + std::to_string(ov_bytes));
            return ov;
        }
        if (b <= bytes) return p;
        if (p) {
            // Kernels queued on any stream the caller used with this problem
            // may still read the old buffer, so growth waits for the whole
            // device.  Calls given a workspace never grow a buffer.
            VSIE_HIP(hipDeviceSynchronize());
            VSIE_HIP(hipFree(p));
        }
        p = nullptr;
        bytes = 0;
        ++g_graph_epoch;
        VSIE_HIP(hipMalloc(&p, b));
        bytes = b;
        return p;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

// The work buffers one call needs (each rounded up to 256 bytes), planned
// before the call from the same layout functions the call uses.
constexpr size_t kWsAlign = 256;
inline size_t ws_round(size_t b) { return (b + kWsAlign - 1) / kWsAlign * kWsAlign; }

struct WsPlan {
    std::vector<std::pair<Scratch *, size_t>> items;
    void need(Scratch &sc, size_t b) {
        for (auto &it : items)
            if (it.first == &sc) {
                it.second = std::max(it.second, b);
                return;
            }
        items.emplace_back(&sc, b);
    }
    size_t total() const {
        size_t t = 0;
        for (const auto &it : items) t += ws_round(it.second);
        return t;
    }
};

// For the duration of one call, the planned buffers live in the caller's
// workspace [ws, ws + bytes): consecutive 256-byte aligned parts in plan
// order.  Without a workspace (ws == NULL) nothing changes.
struct WsScope {
    std::vector<Scratch *> set;
    WsScope(const WsPlan &plan, void *ws, size_t bytes) {
        if (!ws) return;
        if (reinterpret_cast<uintptr_t>(ws) % kWsAlign != 0)
            fail(VSIE_E_INVALID, "workspace must be 256-byte aligned");
        const size_t need = plan.total();
        if (bytes < need)
            fail(VSIE_E_WORKSPACE, "workspace of " + std::to_string(bytes) + " bytes, the call needs " +
                                       std::to_string(need) + " (vsie_workspace_size)");
        // operator graphs hold work-buffer addresses: those captured before
        // this call are not replayed into the workspace, and those captured
        // into it are not replayed after the call (the caller may free it)
        ++g_graph_epoch;
        char *at = static_cast<char *>(ws);
        for (const auto &it : plan.items) {
            it.first->ov = at;
            it.first->ov_bytes = ws_round(it.second);
            it.first->ov_on = true;
            set.push_back(it.first);
            at += ws_round(it.second);
        }
    }
    ~WsScope() {
        if (!set.empty()) ++g_graph_epoch;
        for (Scratch *sc : set) {
            sc->ov = nullptr;
            sc->ov_bytes = 0;
            sc->ov_on = false;
        }
    }
    WsScope(const WsScope &) = delete;
    WsScope &operator=(const WsScope &) = delete;
};

// Grow-only pinned host buffer (hipHostMalloc): device-to-host copies into it
// are truly asynchronous.
struct HostPinned {
    void *p = nullptr;
    size_t bytes = 0;
    void *get(size_t b) {
        if (b <= bytes) return p;
        if (p) VSIE_HIP(hipHostFree(p));
        p = nullptr;
        bytes = 0;
        VSIE_HIP(hipHostMalloc(&p, b, hipHostMallocDefault));
        bytes = b;
        return p;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
};

// Source chunking of one vector pair launch: about target_waves (thread-block,
// chunk) waves to keep every SIMD busy, but chunks of at least kMinChunk
// streamed points.
constexpr int64_t kMinChunk = 256;

void choose_chunks(int64_t n_t, int64_t n_s, int64_t target_waves, int64_t &chunk, int &n_chunks) {
    if (n_s <= 0) {
        chunk = 1;
        n_chunks = 0;
        return;
    }
    const int64_t waves = std::max<int64_t>(1, (n_t + 63) / 64);
    int64_t want = (target_waves + waves - 1) / waves;
    const int64_t max_chunks = std::max<int64_t>(1, n_s / kMinChunk);
    want = std::min<int64_t>(std::max<int64_t>(want, 1), std::min<int64_t>(max_chunks, 4096));
    chunk = (n_s + want - 1) / want;
    n_chunks = static_cast<int>((n_s + chunk - 1) / chunk);
}

}  // namespace vsie

using namespace vsie;

struct vsie_problem {
    int device = 0;
    DeviceMesh m;
    std::vector<double> k0;
    double *d_k0 = nullptr;
    SourceSet G, F;
    int32_t *cf_off = nullptr, *cf_idx = nullptr;  // cell -> adjacent faces (CSR)
    std::vector<void *> owned;  // permanent device allocations
    Scratch partial, chargeG, chargeF, chargeAll, sums_part, grad_work;
    // Krylov workspace
    Scratch V, V2, w, r, ax, h1, tc, nrm, dpart, npart, yv, act, act2, live, kd, kc, xa, axa, rres, brc;
    Scratch defP, defM, defB, defk, lslot;  // deflation of GMRES cycles (gmres_cycle)
    Scratch bh, bg, bsk;  // block GMRES: Hessenberg block column, Gram / inverse factor, slab partials
    Scratch bqk, bbm, bzt;  // block deflation: Q E of each kept space, C^H A V per cycle, coefficients
    Scratch bst;            // block steps of small width: the coefficients of a step, copied at once
    HostPinned hpin;      // per-iteration Hessenberg columns and norms on their way to the host
    int progress = 0;     // vsie_solve_opts::progress of the running solve
    PairProfiler prof;
    vsie_tuning tune{8, 2, 1, 16, 32768, 1, 4, 1, 1, 16, 0};
    // every cell is a single-layer source and the sources are the cells in
    // canonical order (the symmetric cell-cell kernel applies)
    bool g_is_cells = false;
    // the double-layer sources are exactly the faces (no cell has grad alpha)
    bool f_is_faces = false;
    // double-layer sources that are cells (F holds them first, then the faces)
    // and, per 64-cell tile, whether any cell in it has grad alpha
    int64_t f_cells = 0;
    Scratch ctile;
    std::vector<int32_t> ctile_h;  // host copy of the tile flags
    // face-face pairs on the symmetric kernel: tile flags of the faces (all
    // set) and zeros (the faces' single-layer charges and weights)
    Scratch ftile, fzero;
    // host copies of the point positions (fixed at assembly) and of the class
    // lists the device source sets were built from
    std::vector<double> hpx, hpy, hpz;
    std::vector<int32_t> gi_built, fi_built;
    // cached XCD item ranges of the symmetric and cell-face kernels with
    // grad-alpha cells, per precision (valid for group size g)
    struct TRanges {
        int g = -1;
        int64_t sym[9], cf[9];
    } tranges[2];
    double far[3] = {0, 0, 0}, far_step = 1;  // padding points of the tiled kernels
    // dense FP32 off-diagonal operator per frequency (caller-owned memory)
    struct Dense {
        float *A = nullptr;  // real parts; imaginary parts at A + ld n
        int64_t ld = 0;
    };
    std::vector<Dense> dense;
    rocblas_handle blas = nullptr;
    Scratch dense_x, dense_part;
    // captured operator applications (vsie_tuning::graph), keyed by their arguments
    struct OpGraph {
        int f, prec, nrhs;
        bool adjoint;
        const double2 *x;
        int64_t ldx;
        double2 *y;
        int64_t ldy;
        uint64_t epoch;
        hipGraph_t g;
        hipGraphExec_t e;
    };
    std::vector<OpGraph> graphs;
    hipStream_t capture_stream = nullptr;  // graphs are captured here and launched on the caller's stream
    void clear_graphs() {
        for (auto &q : graphs) {
            if (q.e) (void)hipGraphExecDestroy(q.e);
            if (q.g) (void)hipGraphDestroy(q.g);
        }
        graphs.clear();
    }

    template <typename T>
    T *alloc(int64_t count) {
        if (count <= 0) return nullptr;
        void *p = nullptr;
        VSIE_HIP(hipMalloc(&p, sizeof(T) * static_cast<size_t>(count)));
        owned.push_back(p);
        return static_cast<T *>(p);
    }
    template <typename T>
    T *upload(const T *host, int64_t count) {
        if (count <= 0 || host == nullptr) return nullptr;
        T *d = alloc<T>(count);
        VSIE_HIP(hipMemcpy(d, host, sizeof(T) * static_cast<size_t>(count), hipMemcpyHostToDevice));
        return d;
    }
    void free_sources(SourceSet &S) {
        void *ps[] = {S.idx, S.x, S.y, S.z, S.vx, S.vy, S.vz, S.pk, S.pv};
        for (void *q : ps) {
            if (!q) continue;
            auto it = std::find(owned.begin(), owned.end(), q);
            if (it != owned.end()) owned.erase(it);
            (void)hipFree(q);
        }
        S = SourceSet{};
    }
    ~vsie_problem() {
        clear_graphs();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        for (auto &r : prof.recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (hipEvent_t e : prof.pool) (void)hipEventDestroy(e);
        if (blas) (void)rocblas_destroy_handle(blas);
        dense_x.release();
        dense_part.release();
        hpin.release();
        for (void *p : owned) (void)hipFree(p);
        for (Scratch *s : {&partial, &chargeG, &chargeF, &chargeAll, &sums_part, &grad_work, &V, &V2, &w, &r, &ax,
                           &h1, &tc, &nrm, &dpart, &npart, &yv, &act, &act2, &live, &kd, &kc, &xa, &axa, &brc,
                           &rres, &bh, &bg, &bsk, &bqk, &bbm, &bzt, &bst, &defP, &defM, &defB, &defk, &lslot, &ctile,
                           &ftile, &fzero})
            s->release();
    }
};

namespace {

template <typename F>
vsie_status guarded(F &&fn) {
    try {
        fn();
        return VSIE_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return VSIE_E_NOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return VSIE_E_INVALID;
    }
}

inline hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

void require(bool ok, const std::string &msg) {
    if (!ok) fail(VSIE_E_INVALID, msg);
}

void validate_geometry(const vsie_geometry *g, const double *vrho, const double *vc) {
    require(g != nullptr, "geometry is NULL");
    require(g->n_vol >= 0 && g->n_srf >= 0, "negative element count");
    require(g->n_vol + g->n_srf >= 1, "empty problem");
    require(g->n_vol <= INT32_MAX && g->n_srf <= INT32_MAX, "too many elements");
    require(std::isfinite(g->rho0) && g->rho0 > 0 && std::isfinite(g->c0) && g->c0 > 0,
            "rho0 and c0 must be positive");
    const int64_t nv = g->n_vol, ns = g->n_srf;
    if (nv > 0) {
        require(g->vx && g->vy && g->vz && g->vw && g->vdom, "volume arrays must not be NULL");
        require(vrho && vc, "material arrays must not be NULL");
        for (int64_t e = 0; e < nv; ++e) {
            require(std::isfinite(g->vx[e]) && std::isfinite(g->vy[e]) && std::isfinite(g->vz[e]),
                    "non-finite cell centroid at " + std::to_string(e));
            require(g->vw[e] > 0 && std::isfinite(g->vw[e]), "cell volume must be positive at " + std::to_string(e));
            require(g->vdom[e] == 1 || g->vdom[e] == 2, "cell subdomain must be 1 or 2 at " + std::to_string(e));
            require(vrho[e] > 0 && std::isfinite(vrho[e]) && vc[e] > 0 && std::isfinite(vc[e]),
                    "density and sound speed must be positive at cell " + std::to_string(e));
            if (g->vnb)
                for (int a = 0; a < 6; ++a) {
                    const int32_t q = g->vnb[6 * e + a];
                    require(q >= -1 && q < nv && q != e, "bad neighbour index at cell " + std::to_string(e));
                }
            if (g->vgrad_alpha)
                for (int a = 0; a < 3; ++a)
                    require(std::isfinite(g->vgrad_alpha[3 * e + a]), "non-finite grad alpha");
            if (g->vgrad_rho)
                for (int a = 0; a < 3; ++a)
                    require(std::isfinite(g->vgrad_rho[3 * e + a]), "non-finite grad rho");
        }
    }
    if (ns > 0) {
        require(g->sx && g->sy && g->sz && g->snx && g->sny && g->snz && g->sarea && g->siface &&
                    g->scell_in && g->scell_out,
                "surface arrays must not be NULL");
        require(nv > 0, "surface elements need adjacent volume cells");
        for (int64_t q = 0; q < ns; ++q) {
            require(std::isfinite(g->sx[q]) && std::isfinite(g->sy[q]) && std::isfinite(g->sz[q]),
                    "non-finite face centroid at " + std::to_string(q));
            const double nn = g->snx[q] * g->snx[q] + g->sny[q] * g->sny[q] + g->snz[q] * g->snz[q];
            require(std::fabs(std::sqrt(nn) - 1.0) <= 1e-12, "face normal not of unit length at " + std::to_string(q));
            require(g->sarea[q] > 0 && std::isfinite(g->sarea[q]), "face area must be positive");
            require(g->siface[q] == 1 || g->siface[q] == 2, "face interface must be 1 or 2");
            require(g->scell_in[q] >= 0 && g->scell_in[q] < nv, "bad inside cell of face " + std::to_string(q));
            require(g->scell_out[q] >= -1 && g->scell_out[q] < nv, "bad outside cell of face " + std::to_string(q));
            if (g->siface[q] == 1)
                require(g->scell_out[q] == -1, "a Gamma_1 face must have the exterior outside");
            else
                require(g->scell_out[q] >= 0, "a Gamma_2 face needs a cell outside");
        }
    }
}

// Rebuild the class lists (which elements carry a single-layer weight, which a
// v' weight) from the device weights, and pack their coordinates and v'.
// Returns whether anything a captured operator graph holds changed: a class
// list (its device arrays and counts) or the grad-alpha tile flags (and with
// them the XCD ranges of the kernels).  The weights are rewritten in place.
bool build_sources(vsie_problem *p) {
    const int64_t n = p->m.n;
    const int nf = static_cast<int>(p->k0.size());
    std::vector<double> sp(static_cast<size_t>(n) * nf), vp(3 * static_cast<size_t>(n));
    VSIE_HIP(hipMemcpy(sp.data(), p->m.sp, sizeof(double) * sp.size(), hipMemcpyDeviceToHost));
    VSIE_HIP(hipMemcpy(vp.data(), p->m.vpx, sizeof(double) * n, hipMemcpyDeviceToHost));
    VSIE_HIP(hipMemcpy(vp.data() + n, p->m.vpy, sizeof(double) * n, hipMemcpyDeviceToHost));
    VSIE_HIP(hipMemcpy(vp.data() + 2 * n, p->m.vpz, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (static_cast<int64_t>(p->hpx.size()) != n) {
        p->hpx.resize(n);
        p->hpy.resize(n);
        p->hpz.resize(n);
        VSIE_HIP(hipMemcpy(p->hpx.data(), p->m.px, sizeof(double) * n, hipMemcpyDeviceToHost));
        VSIE_HIP(hipMemcpy(p->hpy.data(), p->m.py, sizeof(double) * n, hipMemcpyDeviceToHost));
        VSIE_HIP(hipMemcpy(p->hpz.data(), p->m.pz, sizeof(double) * n, hipMemcpyDeviceToHost));
    }
    const std::vector<double> &px = p->hpx, &py = p->hpy, &pz = p->hpz;
    for (double v : sp) require(std::isfinite(v), "non-finite single-layer weight");
    for (double v : vp) require(std::isfinite(v), "non-finite double-layer weight");
    std::vector<int32_t> gi, fi;
    for (int64_t e = 0; e < n; ++e) {
        bool g = false;
        for (int f = 0; f < nf; ++f) g = g || sp[static_cast<size_t>(f) * n + e] != 0.0;
        if (g) gi.push_back(static_cast<int32_t>(e));
        if (vp[e] != 0.0 || vp[n + e] != 0.0 || vp[2 * n + e] != 0.0) fi.push_back(static_cast<int32_t>(e));
    }
    // the class lists of the previous materials: G keeps its device arrays
    // (positions only), F its positions with the new v'
    const bool keep_g = !gi.empty() && gi == p->gi_built && p->G.idx;
    const bool keep_f = !fi.empty() && fi == p->fi_built && p->F.idx;
    if (!keep_g) p->free_sources(p->G);
    if (!keep_f) p->free_sources(p->F);
    // padding point of the matrix-core layout: farther than the extent of the
    // mesh from every point (its pairs are finite and meet zero charges)
    double lo3[3] = {px[0], py[0], pz[0]}, hi3[3] = {px[0], py[0], pz[0]};
    for (int64_t e = 0; e < n; ++e) {
        const double q[3] = {px[e], py[e], pz[e]};
        for (int d = 0; d < 3; ++d) {
            lo3[d] = std::min(lo3[d], q[d]);
            hi3[d] = std::max(hi3[d], q[d]);
        }
    }
    const double ext = std::max({hi3[0] - lo3[0], hi3[1] - lo3[1], hi3[2] - lo3[2]}) + 1.0;
    for (int d = 0; d < 3; ++d) p->far[d] = hi3[d] + ext;
    p->far_step = ext;
    p->g_is_cells = static_cast<int64_t>(gi.size()) == p->m.n_vol && p->m.n_vol > 0;
    p->f_is_faces = static_cast<int64_t>(fi.size()) == p->m.n_srf && p->m.n_srf > 0 && fi[0] == p->m.n_vol;
    p->f_cells = 0;
    for (int32_t e : fi) p->f_cells += e < p->m.n_vol ? 1 : 0;
    bool flags_changed = true;
    {
        const int64_t tiles = (p->m.n_vol + 63) / 64;
        std::vector<int32_t> flag(static_cast<size_t>(std::max<int64_t>(1, tiles)), 0);
        for (int64_t e = 0; e < p->m.n_vol; ++e)
            if (vp[e] != 0.0 || vp[n + e] != 0.0 || vp[2 * n + e] != 0.0) flag[static_cast<size_t>(e / 64)] = 1;
        flags_changed = flag != p->ctile_h;
        void *d = p->ctile.get(sizeof(int32_t) * flag.size());
        VSIE_HIP(hipMemcpy(d, flag.data(), sizeof(int32_t) * flag.size(), hipMemcpyHostToDevice));
        p->ctile_h = flag;
        if (flags_changed)
            for (auto &r : p->tranges) r.g = -1;
    }
    if (p->m.n_srf > 0 && !p->ftile.p) {
        const std::vector<int32_t> ones(static_cast<size_t>((p->m.n_srf + 63) / 64), 1);
        void *d = p->ftile.get(sizeof(int32_t) * ones.size());
        VSIE_HIP(hipMemcpy(d, ones.data(), sizeof(int32_t) * ones.size(), hipMemcpyHostToDevice));
        void *z = p->fzero.get(sizeof(double2) * static_cast<size_t>(p->m.n_srf));
        VSIE_HIP(hipMemset(z, 0, sizeof(double2) * static_cast<size_t>(p->m.n_srf)));
    }
    auto fill = [&](SourceSet &S, const std::vector<int32_t> &ix, bool with_v) {
        S.count = static_cast<int64_t>(ix.size());
        if (S.count == 0) return;
        std::vector<double> a(S.count), b(S.count), c(S.count);
        std::vector<double4> pk(S.count + kMfmaPad), pv(S.count + kMfmaPad);
        for (int64_t j = 0; j < S.count; ++j) {
            a[j] = px[ix[j]];
            b[j] = py[ix[j]];
            c[j] = pz[ix[j]];
            pk[j] = make_double4(a[j], b[j], c[j], 0.0);
        }
        for (int t = 0; t < kMfmaPad; ++t) {
            pk[S.count + t] = make_double4(hi3[0] + ext, hi3[1] + ext, hi3[2] + ext, 0.0);
            pv[S.count + t] = make_double4(0.0, 0.0, 0.0, 0.0);
        }
        S.idx = p->upload(ix.data(), S.count);
        S.x = p->upload(a.data(), S.count);
        S.y = p->upload(b.data(), S.count);
        S.z = p->upload(c.data(), S.count);
        S.pk = p->upload(pk.data(), S.count + kMfmaPad);
        if (!with_v) return;
        std::vector<double> va(S.count), vb(S.count), vc(S.count);
        for (int64_t j = 0; j < S.count; ++j) {
            va[j] = vp[ix[j]];
            vb[j] = vp[n + ix[j]];
            vc[j] = vp[2 * n + ix[j]];
            pv[j] = make_double4(va[j], vb[j], vc[j], 0.0);
        }
        S.vx = p->upload(va.data(), S.count);
        S.vy = p->upload(vb.data(), S.count);
        S.vz = p->upload(vc.data(), S.count);
        S.pv = p->upload(pv.data(), S.count + kMfmaPad);
    };
    if (!keep_g) fill(p->G, gi, false);
    if (keep_f) {
        // same F points: only their v' changed (queued products that read
        // the old values finish first)
        VSIE_HIP(hipDeviceSynchronize());
        const int64_t cnt = p->F.count;
        std::vector<double> va(cnt), vb(cnt), vc(cnt);
        std::vector<double4> pv(cnt + kMfmaPad, make_double4(0.0, 0.0, 0.0, 0.0));
        for (int64_t j = 0; j < cnt; ++j) {
            va[j] = vp[fi[j]];
            vb[j] = vp[n + fi[j]];
            vc[j] = vp[2 * n + fi[j]];
            pv[j] = make_double4(va[j], vb[j], vc[j], 0.0);
        }
        VSIE_HIP(hipMemcpy(p->F.vx, va.data(), sizeof(double) * cnt, hipMemcpyHostToDevice));
        VSIE_HIP(hipMemcpy(p->F.vy, vb.data(), sizeof(double) * cnt, hipMemcpyHostToDevice));
        VSIE_HIP(hipMemcpy(p->F.vz, vc.data(), sizeof(double) * cnt, hipMemcpyHostToDevice));
        VSIE_HIP(hipMemcpy(p->F.pv, pv.data(), sizeof(double4) * (cnt + kMfmaPad), hipMemcpyHostToDevice));
    } else {
        fill(p->F, fi, true);
    }
    p->gi_built = gi;
    p->fi_built = fi;
    return !keep_g || !keep_f || flags_changed;
}

void check_problem(const vsie_problem *p, int32_t f) {
    require(p != nullptr, "problem handle is NULL");
    require(f >= 0 && f < static_cast<int32_t>(p->k0.size()), "frequency index out of range");
}

void check_vec(const double *v, int64_t ld, int64_t n, const char *name) {
    require(v != nullptr, std::string(name) + " is NULL");
    require(ld >= n, std::string("leading dimension of ") + name + " is smaller than n");
}

size_t csize(vsie_precision prec) { return prec == VSIE_FP64 ? sizeof(double2) : sizeof(float2); }

// Chunking and work-buffer sizes of apply_forward_block.
struct FwdBlockLayout {
    int64_t chG, chF;
    int ncG, ncF;
    size_t part, qG, qF;
};
FwdBlockLayout fwd_block_layout(const vsie_problem *p, vsie_precision prec, int nrhs) {
    FwdBlockLayout L;
    const int64_t n = p->m.n;
    choose_chunks(n, p->G.count, p->tune.vec_target_waves, L.chG, L.ncG);
    choose_chunks(n, p->F.count, p->tune.vec_target_waves, L.chF, L.ncF);
    L.part = sizeof(double2) * static_cast<size_t>(std::max(1, L.ncG + L.ncF)) * nrhs * n;
    L.qG = csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->G.count)) * nrhs;
    L.qF = csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->F.count)) * nrhs;
    return L;
}
void plan_forward_block(vsie_problem *p, vsie_precision prec, int nrhs, WsPlan &pl) {
    const FwdBlockLayout L = fwd_block_layout(p, prec, nrhs);
    pl.need(p->partial, L.part);
    pl.need(p->chargeG, L.qG);
    pl.need(p->chargeF, L.qF);
}

// y = A_f x (forward operator) for at most kMaxRhsPerLaunch columns.
void apply_forward_block(vsie_problem *p, int f, vsie_precision prec, int nrhs, const double2 *x,
                         int64_t ldx, double2 *y, int64_t ldy, hipStream_t s) {
    const int64_t n = p->m.n;
    const FwdBlockLayout L = fwd_block_layout(p, prec, nrhs);
    const int64_t chG = L.chG, chF = L.chF;
    const int ncG = L.ncG, ncF = L.ncF;
    const int n_parts = ncG + ncF;
    double2 *part = static_cast<double2 *>(p->partial.get(L.part));
    void *qG = p->chargeG.get(L.qG);
    void *qF = p->chargeF.get(L.qF);
    const double *spf = p->m.sp + static_cast<int64_t>(f) * n;
    launch_pack_charges(kClassG, prec, p->G, spf, nrhs, x, ldx, false, qG, s);
    launch_pack_charges(kClassF, prec, p->F, spf, nrhs, x, ldx, false, qF, s);
    const double k = p->k0[f];
    if (ncG > 0) {
        PairJob J{PAIR_FWD_G, prec, n, p->m.px, p->m.py, p->m.pz, {}, p->G.count,
                  p->G.x, p->G.y, p->G.z, {}, qG, p->G.count, nrhs, chG, ncG, k,
                  part, static_cast<int64_t>(nrhs) * n, SELF_STREAM_IDX, p->G.idx};
        launch_pairs(J, s, &p->prof);
    }
    if (ncF > 0) {
        PairJob J{PAIR_FWD_F, prec, n, p->m.px, p->m.py, p->m.pz, {}, p->F.count,
                  p->F.x, p->F.y, p->F.z, {p->F.vx, p->F.vy, p->F.vz},
                  qF, p->F.count, nrhs, chF, ncF, k,
                  part + static_cast<int64_t>(ncG) * nrhs * n, static_cast<int64_t>(nrhs) * n,
                  SELF_STREAM_IDX, p->F.idx};
        launch_pairs(J, s, &p->prof);
    }
    launch_reduce_partials(n, nrhs, n_parts, part, p->m.diag + static_cast<int64_t>(f) * n, false, x,
                           ldx, y, ldy, nullptr, s);
}

// The once-per-pair kernels' slot partials, four arrays of float2 (FP32
// operator) or double2 entries, then a double2 tail for the one-sided chunk
// partials; every array starts on a 256-byte boundary.
struct SlotBuffers {
    void *s[4];
    double2 *tail;
};

// Bytes of the slot buffers and the offsets of their five parts.
size_t slot_layout(vsie_precision prec, std::initializer_list<int64_t> counts, int64_t tail, size_t off[5]) {
    if (counts.size() != 4) fail(VSIE_E_INVALID, "slot buffers: four slot arrays expected");
    const size_t es = prec == VSIE_FP32 ? sizeof(float2) : sizeof(double2);
    size_t at = 0;
    int i = 0;
    for (int64_t c : counts) {
        off[i++] = at;
        at += ws_round(es * static_cast<size_t>(c));
    }
    off[4] = at;
    at += sizeof(double2) * static_cast<size_t>(tail);
    return std::max<size_t>(256, at);
}

SlotBuffers slot_buffers(vsie_problem *p, vsie_precision prec, std::initializer_list<int64_t> counts,
                         int64_t tail) {
    size_t off[5];
    char *base = static_cast<char *>(p->partial.get(slot_layout(prec, counts, tail, off)));
    return SlotBuffers{{base + off[0], base + off[1], base + off[2], base + off[3]},
                       reinterpret_cast<double2 *>(base + off[4])};
}

// y = A_f x for one right-hand side with the cell-cell single layer evaluated
// once per unordered pair: the symmetric kernel for cell targets, the vector
// kernel for face targets (no face is a single-layer source, so nothing is
// masked there), the double layers over every target, one reduction.
// The same with the cell-face and face-face pairs once per pair as well:
// symmetric cell-cell single layer (and adjoint double layer of grad-alpha
// cells), cell-face kernel (single layer at faces, double layers at cells),
// face-face double layers on the symmetric kernel, one reduction.

// The once-per-pair kernels write one partial per point and partner group:
// about n_cells^2 / (64 G) for the cell-cell pairs.  The group size G is the
// tuned one, doubled (up to 8) while the partials would exceed
// kSymPartialSoft at the FP64 size: meshes that large have items enough for
// bigger groups (at c1 size, groups of 8 leave too few items to fill the
// chip).  Above kSymPartialCap (counted at the FP64 size) the one-sided
// kernels are used.
constexpr double kSymPartialSoft = 8.0 * (1 << 30);
constexpr double kSymPartialCap = 64.0 * (1 << 30);
constexpr int kFaceGroups = 1;

// slot partials of a one-column product with cell groups of g tiles
double sym_partial_entries(const vsie_problem *p, int g) {
    const int64_t nv = p->m.n_vol, ns = p->m.n - nv;
    double e = static_cast<double>(sym_slots(nv, g)) * nv;
    if (p->tune.cell_face && ns > 0)
        e += static_cast<double>(cf_groups(ns)) * nv + static_cast<double>(cf_groups(nv)) * ns +
             static_cast<double>(sym_slots(ns, kFaceGroups)) * ns;
    return e;
}

int sym_group(const vsie_problem *p) {
    int g = p->tune.sym_groups;
    while (g > 0 && g < 8 && sym_partial_entries(p, g) * sizeof(double2) > kSymPartialSoft) g *= 2;
    return g;
}

// XCD item ranges of the once-per-pair kernels with grad-alpha cells, cached
// per precision and group size.  Issue cycles per pair of the grad-alpha loops
// relative to the single-layer ones (counted in the compiled loops):
// symmetric kernel 1.53 (FP32) and 1.42 (FP64), cell-face kernel 1.17 and 1.42.
const vsie_problem::TRanges &t_ranges(vsie_problem *p, vsie_precision prec) {
    const int g = sym_group(p);
    vsie_problem::TRanges &tr = p->tranges[prec == VSIE_FP32 ? 1 : 0];
    if (tr.g != g) {
        const bool f32 = prec == VSIE_FP32;
        sym_cost_ranges(p->m.n_vol, g, p->ctile_h, f32 ? 1.53 : 1.42, tr.sym);
        cf_cost_ranges(p->m.n_vol, p->m.n - p->m.n_vol, p->ctile_h, f32 ? 1.17 : 1.42, tr.cf);
        tr.g = g;
    }
    return tr;
}

// Face-face double layers once per pair: the symmetric kernel's grad-alpha
// loop over the faces, with the faces' v' (zero where a face carries no jump)
// and zero single-layer charges (forward) or weights (adjoint); every face
// tile is flagged.  Group size 1 (one tile pair per item, kFaceGroups)
// gives enough work items for the few face tiles: on 212 face tiles
// 0.140 ms in FP32, against 0.159 ms with groups of 2 and 0.255 ms with
// groups of 4.

SymJob face_face_job(vsie_problem *p, vsie_precision prec, double k, const void *q, const double2 *xf, void *part) {
    const int64_t nv = p->m.n_vol, ns = p->m.n - nv;
    SymJob J{prec, ns, p->m.px + nv, p->m.py + nv, p->m.pz + nv, q, k, {p->far[0], p->far[1], p->far[2]},
             p->far_step, kFaceGroups, part, ns};
    J.vx = p->m.vpx + nv;
    J.vy = p->m.vpy + nv;
    J.vz = p->m.vpz + nv;
    J.xv = xf;
    J.tile_t = static_cast<const int32_t *>(p->ftile.p);
    J.prof_kind = 18;
    return J;
}

// Slot counts of the once-per-pair products with the cell-face kernel: the
// symmetric cell-cell slots per cell, the face-group slots per cell, the
// cell-group slots per face and the face-face slots per face.
struct CfCounts {
    int64_t slots, cs, fs, ffs;
};
CfCounts cf_counts(const vsie_problem *p) {
    const int64_t nv = p->m.n_vol, ns = p->m.n - nv;
    return CfCounts{sym_slots(nv, sym_group(p)), cf_groups(ns), cf_groups(nv),
                    ns > 0 ? sym_slots(ns, kFaceGroups) : 0};
}
size_t cf_slot_bytes(const vsie_problem *p, vsie_precision prec) {
    const int64_t nv = p->m.n_vol, ns = p->m.n - nv;
    const CfCounts c = cf_counts(p);
    size_t off[5];
    return slot_layout(prec, {c.slots * nv, c.cs * nv, c.fs * ns, c.ffs * ns}, 0, off);
}
void plan_forward_cf(vsie_problem *p, vsie_precision prec, WsPlan &pl) {
    pl.need(p->partial, cf_slot_bytes(p, prec));
    pl.need(p->chargeG, csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->G.count)));
}

void apply_forward_cf(vsie_problem *p, int f, vsie_precision prec, const double2 *x, double2 *y, hipStream_t s) {
    const int64_t n = p->m.n, nv = p->m.n_vol, ns = n - nv;
    const int g = sym_group(p);
    const CfCounts cc = cf_counts(p);
    const int64_t slots = cc.slots, cs = cc.cs, fs = cc.fs, ffs = cc.ffs;
    const SlotBuffers sb = slot_buffers(p, prec, {slots * nv, cs * nv, fs * ns, ffs * ns}, 0);
    void *psym = sb.s[0], *pc = sb.s[1], *pf = sb.s[2], *pff = sb.s[3];
    // the single-layer charges -s' x of the cells; the double layers take the
    // raw values x
    void *qG = p->chargeG.get(csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->G.count)));
    const double *spf = p->m.sp + static_cast<int64_t>(f) * n;
    launch_pack_charges(kClassG, prec, p->G, spf, 1, x, n, false, qG, s);
    const double k = p->k0[f];
    const bool t = p->f_cells > 0;
    const int32_t *tiles_t = static_cast<const int32_t *>(p->ctile.p);
    SymJob J{prec, nv, p->m.px, p->m.py, p->m.pz, qG, k, {p->far[0], p->far[1], p->far[2]}, p->far_step, g, psym, nv};
    if (t) {
        const vsie_problem::TRanges &tr = t_ranges(p, prec);
        J.vx = p->m.vpx;
        J.vy = p->m.vpy;
        J.vz = p->m.vpz;
        J.xv = x;
        J.tile_t = tiles_t;
        J.xr = tr.sym;
    }
    launch_sym(J, s, &p->prof);
    if (ns > 0) {
        CfJob C{prec, nv, ns, p->m.px, p->m.py, p->m.pz, p->m.vpx + nv, p->m.vpy + nv, p->m.vpz + nv, qG, x + nv, k,
                {p->far[0], p->far[1], p->far[2]}, p->far_step, pc, pf};
        if (t) {
            C.cvx = p->m.vpx;
            C.cvy = p->m.vpy;
            C.cvz = p->m.vpz;
            C.xc = x;
            C.ctile_t = tiles_t;
            C.xr = t_ranges(p, prec).cf;
        }
        launch_cf(C, s, &p->prof);
        const SymJob Jf = face_face_job(p, prec, k, p->fzero.p, x + nv, pff);
        launch_sym(Jf, s, &p->prof);
    }
    const bool f32 = prec == VSIE_FP32;
    launch_cf_reduce(n, nv, f32, static_cast<int>(slots), psym, static_cast<int>(cs), pc, static_cast<int>(fs), pf,
                     static_cast<int>(ffs), pff, f32, p->m.diag + static_cast<int64_t>(f) * n, x, y, s);
}

// Chunking of the one-sided parts of apply_forward_sym without the
// cell-face kernel (single layer at the faces, double layers everywhere).
struct SymLayout {
    int64_t slots, chGf = 1, chF = 1;
    int ncGf = 0, ncF = 0;
    size_t part;
};
SymLayout sym_layout(const vsie_problem *p, vsie_precision prec) {
    const int64_t n = p->m.n, nv = p->m.n_vol, ns = n - nv;
    SymLayout L;
    L.slots = sym_slots(nv, sym_group(p));
    if (ns > 0) choose_chunks(ns, p->G.count, p->tune.vec_target_waves, L.chGf, L.ncGf);
    choose_chunks(n, p->F.count, p->tune.vec_target_waves, L.chF, L.ncF);
    size_t off[5];
    L.part = slot_layout(prec, {L.slots * nv, 0, 0, 0}, static_cast<int64_t>(L.ncGf) * ns + static_cast<int64_t>(L.ncF) * n,
                         off);
    return L;
}
void plan_forward_sym(vsie_problem *p, vsie_precision prec, WsPlan &pl) {
    if (p->tune.cell_face) {
        plan_forward_cf(p, prec, pl);
        return;
    }
    pl.need(p->partial, sym_layout(p, prec).part);
    pl.need(p->chargeG, csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->G.count)));
    pl.need(p->chargeF, csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->F.count)));
}

void apply_forward_sym(vsie_problem *p, int f, vsie_precision prec, const double2 *x, double2 *y,
                       hipStream_t s) {
    if (p->tune.cell_face) {
        apply_forward_cf(p, f, prec, x, y, s);
        return;
    }
    const int64_t n = p->m.n, nv = p->m.n_vol, ns = n - nv;
    const int g = sym_group(p);
    const SymLayout L = sym_layout(p, prec);
    const int64_t slots = L.slots, chGf = L.chGf, chF = L.chF;
    const int ncGf = L.ncGf, ncF = L.ncF;
    const SlotBuffers sb = slot_buffers(p, prec, {slots * nv, 0, 0, 0},
                                        static_cast<int64_t>(ncGf) * ns + static_cast<int64_t>(ncF) * n);
    void *psym = sb.s[0];
    double2 *pface = sb.tail, *pF = pface + static_cast<int64_t>(ncGf) * ns;
    void *qG = p->chargeG.get(csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->G.count)));
    void *qF = p->chargeF.get(csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->F.count)));
    const double *spf = p->m.sp + static_cast<int64_t>(f) * n;
    launch_pack_both(prec, p->G, p->F, spf, 1, x, n, false, qG, qF, s);
    const double k = p->k0[f];
    SymJob J{prec, nv, p->m.px, p->m.py, p->m.pz, qG, k, {p->far[0], p->far[1], p->far[2]}, p->far_step, g, psym, nv};
    launch_sym(J, s, &p->prof);
    if (ncGf > 0) {
        PairJob Jf{PAIR_FWD_G, prec, ns, p->m.px + nv, p->m.py + nv, p->m.pz + nv, {}, p->G.count,
                   p->G.x, p->G.y, p->G.z, {}, qG, p->G.count, 1, chGf, ncGf, k, pface, ns, SELF_DISJOINT, nullptr};
        launch_pairs(Jf, s, &p->prof);
    }
    if (ncF > 0) {
        PairJob JF{PAIR_FWD_F, prec, n, p->m.px, p->m.py, p->m.pz, {}, p->F.count,
                   p->F.x, p->F.y, p->F.z, {p->F.vx, p->F.vy, p->F.vz}, qF, p->F.count, 1, chF, ncF, k,
                   pF, n, SELF_STREAM_IDX, p->F.idx};
        launch_pairs(JF, s, &p->prof);
    }
    launch_sym_reduce(n, nv, static_cast<int>(slots), psym, prec == VSIE_FP32, nv, ncGf, pface, ncF, pF,
                      p->m.diag + static_cast<int64_t>(f) * n, x, y, s);
}

bool use_sym(const vsie_problem *p, int nrhs) {
    if (nrhs != 1 || p->tune.sym_groups <= 0 || !p->g_is_cells) return false;
    return sym_partial_entries(p, sym_group(p)) * sizeof(double2) <= kSymPartialCap;
}

void plan_forward(vsie_problem *p, vsie_precision prec, int nrhs, WsPlan &pl) {
    if (use_sym(p, nrhs)) {
        plan_forward_sym(p, prec, pl);
        return;
    }
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPerLaunch) plan_forward_block(p, prec, std::min(kMaxRhsPerLaunch, nrhs - r0), pl);
}

void apply_forward(vsie_problem *p, int f, vsie_precision prec, int nrhs, const double2 *x,
                   int64_t ldx, double2 *y, int64_t ldy, hipStream_t s) {
    if (use_sym(p, nrhs)) {
        apply_forward_sym(p, f, prec, x, y, s);
        return;
    }
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPerLaunch) {
        const int blk = std::min(kMaxRhsPerLaunch, nrhs - r0);
        apply_forward_block(p, f, prec, blk, x + static_cast<int64_t>(r0) * ldx, ldx,
                            y + static_cast<int64_t>(r0) * ldy, ldy, s);
    }
}

// y = A_f^H x for at most kMaxRhsPerLaunch columns:
// (A^H x)_j = conj(A_jj) x_j + sum_{i != j} conj(A_ij) x_i, evaluated per source
// class with the roles of targets and sources exchanged.
struct AdjBlockLayout {
    int64_t chG = 1, chF = 1;
    int ncG = 0, ncF = 0;
    size_t q, part;
};
AdjBlockLayout adj_block_layout(const vsie_problem *p, vsie_precision prec, int nrhs) {
    const int64_t n = p->m.n;
    AdjBlockLayout L;
    if (p->G.count > 0) choose_chunks(p->G.count, n, p->tune.vec_target_waves, L.chG, L.ncG);
    if (p->F.count > 0) choose_chunks(p->F.count, n, p->tune.vec_target_waves, L.chF, L.ncF);
    const size_t need = std::max(static_cast<size_t>(L.ncG) * p->G.count, static_cast<size_t>(L.ncF) * p->F.count);
    L.q = csize(prec) * static_cast<size_t>(n) * nrhs;
    L.part = sizeof(double2) * std::max<size_t>(1, need) * nrhs;
    return L;
}
void plan_adjoint_block(vsie_problem *p, vsie_precision prec, int nrhs, WsPlan &pl) {
    const AdjBlockLayout L = adj_block_layout(p, prec, nrhs);
    pl.need(p->chargeAll, L.q);
    pl.need(p->partial, L.part);
}

void apply_adjoint_block(vsie_problem *p, int f, vsie_precision prec, int nrhs, const double2 *x,
                         int64_t ldx, double2 *y, int64_t ldy, hipStream_t s) {
    const int64_t n = p->m.n;
    const AdjBlockLayout L = adj_block_layout(p, prec, nrhs);
    void *q = p->chargeAll.get(L.q);
    launch_pack_plain(prec, n, nrhs, x, ldx, true, q, s);
    // y = conj(diag) x
    launch_reduce_partials(n, nrhs, 0, nullptr, p->m.diag + static_cast<int64_t>(f) * n, true, x, ldx,
                           y, ldy, nullptr, s);
    const double k = p->k0[f];
    const double *spf = p->m.sp + static_cast<int64_t>(f) * n;
    const int64_t chG = L.chG, chF = L.chF;
    const int ncG = L.ncG, ncF = L.ncF;
    double2 *part = static_cast<double2 *>(p->partial.get(L.part));
    if (ncG > 0) {
        PairJob J{PAIR_FWD_G, prec, p->G.count, p->G.x, p->G.y, p->G.z, {}, n,
                  p->m.px, p->m.py, p->m.pz, {}, q, n, nrhs, chG, ncG, k, part,
                  static_cast<int64_t>(nrhs) * p->G.count, SELF_THREAD_IDX, p->G.idx};
        launch_pairs(J, s, &p->prof);
        launch_scatter_conj(p->G.count, p->G.idx, spf, nrhs, ncG, part, y, ldy, s);
    }
    if (ncF > 0) {
        PairJob J{PAIR_ADJ_F, prec, p->F.count, p->F.x, p->F.y, p->F.z,
                  {p->F.vx, p->F.vy, p->F.vz}, n,
                  p->m.px, p->m.py, p->m.pz, {}, q, n, nrhs, chF, ncF, k, part,
                  static_cast<int64_t>(nrhs) * p->F.count, SELF_THREAD_IDX, p->F.idx};
        launch_pairs(J, s, &p->prof);
        launch_scatter_conj(p->F.count, p->F.idx, nullptr, nrhs, ncF, part, y, ldy, s);
    }
}

// One-column adjoint with the once-per-pair kernels, when every cell is a
// single-layer source.  With mu = conj(lambda):
// (A^H lambda)_j = conj(d_j) lambda_j + conj(S_j), where a cell's S_j sums
// (-s'_j e_ij + F_ij (x_i - x_j).v'_j) mu_i over the other cells (symmetric
// kernel) and the faces (cell-face kernel), and a face's S_j sums its double
// layer F_ij (x_i - x_j).v'_j mu_i over the cells (cell-face kernel) and the
// faces (one-sided).  Without grad-alpha cells the cells' sums are of e_ij mu_i
// alone and -s'_j is applied in the reduction.
bool adjoint_sym_ok(const vsie_problem *p, int nrhs) {
    return use_sym(p, nrhs) && p->tune.cell_face;
}

void plan_adjoint_sym(vsie_problem *p, vsie_precision prec, WsPlan &pl) {
    pl.need(p->partial, cf_slot_bytes(p, prec));
    pl.need(p->chargeAll, csize(prec) * static_cast<size_t>(p->m.n));
}

void apply_adjoint_sym(vsie_problem *p, int f, vsie_precision prec, const double2 *x, double2 *y, hipStream_t s) {
    const int64_t n = p->m.n, nv = p->m.n_vol, ns = n - nv;
    const int g = sym_group(p);
    const CfCounts cc = cf_counts(p);
    const int64_t slots = cc.slots, cs = cc.cs, fs = cc.fs, ffs = cc.ffs;
    const SlotBuffers sb = slot_buffers(p, prec, {slots * nv, cs * nv, fs * ns, ffs * ns}, 0);
    void *psym = sb.s[0], *pc = sb.s[1], *pf = sb.s[2], *pff = sb.s[3];
    void *q = p->chargeAll.get(csize(prec) * static_cast<size_t>(n));
    launch_pack_plain(prec, n, 1, x, n, true, q, s);
    const void *qf = static_cast<const char *>(q) + csize(prec) * static_cast<size_t>(nv);
    const double k = p->k0[f];
    const double *spf = p->m.sp + static_cast<int64_t>(f) * n;
    const bool t = p->f_cells > 0;
    const int32_t *tiles_t = static_cast<const int32_t *>(p->ctile.p);
    SymJob J{prec, nv, p->m.px, p->m.py, p->m.pz, q, k, {p->far[0], p->far[1], p->far[2]}, p->far_step, g, psym, nv};
    if (t) {
        J.vx = p->m.vpx;
        J.vy = p->m.vpy;
        J.vz = p->m.vpz;
        J.xv = x;
        J.tile_t = tiles_t;
        J.xr = t_ranges(p, prec).sym;
        J.adj = true;
        J.sw = spf;
    }
    launch_sym(J, s, &p->prof);
    if (ns > 0) {
        CfJob C{prec, nv, ns, p->m.px, p->m.py, p->m.pz, p->m.vpx + nv, p->m.vpy + nv, p->m.vpz + nv, q, nullptr, k,
                {p->far[0], p->far[1], p->far[2]}, p->far_step, pc, pf};
        C.adj = true;
        C.qfa = qf;
        if (t) {
            C.cvx = p->m.vpx;
            C.cvy = p->m.vpy;
            C.cvz = p->m.vpz;
            C.xc = x;
            C.ctile_t = tiles_t;
            C.xr = t_ranges(p, prec).cf;
            C.sw = spf;
        }
        launch_cf(C, s, &p->prof);
        // faces' charges mu, zero single-layer weights: each face target sums
        // its own double layer F (x_i - x_j).v'_j mu_i
        SymJob Jf = face_face_job(p, prec, k, qf, x + nv, pff);
        Jf.adj = true;
        Jf.sw = static_cast<const double *>(p->fzero.p);
        launch_sym(Jf, s, &p->prof);
    }
    const bool f32 = prec == VSIE_FP32;
    launch_cf_reduce(n, nv, f32, static_cast<int>(slots), psym, static_cast<int>(cs), pc, static_cast<int>(fs), pf,
                     static_cast<int>(ffs), pff, f32, p->m.diag + static_cast<int64_t>(f) * n, x, y, s, true,
                     t ? nullptr : spf);
}

void plan_adjoint(vsie_problem *p, vsie_precision prec, int nrhs, WsPlan &pl) {
    if (nrhs == 1 && adjoint_sym_ok(p, nrhs)) {
        plan_adjoint_sym(p, prec, pl);
        return;
    }
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPerLaunch) plan_adjoint_block(p, prec, std::min(kMaxRhsPerLaunch, nrhs - r0), pl);
}

void apply_adjoint(vsie_problem *p, int f, vsie_precision prec, int nrhs, const double2 *x,
                   int64_t ldx, double2 *y, int64_t ldy, hipStream_t s) {
    if (nrhs == 1 && adjoint_sym_ok(p, nrhs)) {
        apply_adjoint_sym(p, f, prec, x, y, s);
        return;
    }
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPerLaunch) {
        const int blk = std::min(kMaxRhsPerLaunch, nrhs - r0);
        apply_adjoint_block(p, f, prec, blk, x + static_cast<int64_t>(r0) * ldx, ldx,
                            y + static_cast<int64_t>(r0) * ldy, ldy, s);
    }
}

// FP32 product with the assembled operator of frequency f: y = d x + A x (or
// conj(d) x + A^H x), in passes of at most kDenseCols columns on the matrix
// cores (dense_kernels.hip): FP32 sums over slabs of kDenseSlab sources,
// added in FP64 in slab order with the FP64 diagonal.
void plan_dense(vsie_problem *p, int nrhs, WsPlan &pl) {
    const int64_t n = p->m.n;
    const int blk = std::min(nrhs, kDenseCols);
    const int64_t slabs = (n + kDenseSlab - 1) / kDenseSlab;
    pl.need(p->dense_x, sizeof(float) * 2 * static_cast<size_t>(dense_npad(n)) * kDenseCols);
    pl.need(p->dense_part, sizeof(double2) * static_cast<size_t>(slabs * blk * n));
}

void apply_dense(vsie_problem *p, int f, bool adjoint, int nrhs, const double2 *x, int64_t ldx,
                 double2 *y, int64_t ldy, hipStream_t s) {
    const int64_t n = p->m.n;
    const auto &D = p->dense[f];
    const int64_t slabs = (n + kDenseSlab - 1) / kDenseSlab;
    float *xp = static_cast<float *>(
        p->dense_x.get(sizeof(float) * 2 * static_cast<size_t>(dense_npad(n)) * kDenseCols));
    for (int r0 = 0; r0 < nrhs; r0 += kDenseCols) {
        const int blk = std::min(kDenseCols, nrhs - r0);
        double2 *part = static_cast<double2 *>(p->dense_part.get(sizeof(double2) * static_cast<size_t>(slabs * blk * n)));
        const DenseJob J{adjoint, p->tune.mfma_3m != 0, n, D.A, D.A + D.ld * n, D.ld, blk,
                         x + static_cast<int64_t>(r0) * ldx, ldx, xp, part, p->m.diag + static_cast<int64_t>(f) * n,
                         y + static_cast<int64_t>(r0) * ldy, ldy};
        launch_dense_product(J, s, &p->prof);
    }
}

// FP32 forward products on the matrix cores for the nf frequencies f0 ..:
// y_t = A_{f0+t} x_t, x_t = x + t xfs, y_t = y + t yfs, at most kMfmaMaxCols
// columns per pass.  Each source class is one launch over all
// frequencies; the partial sums of every frequency are then reduced with its
// FP64 diagonal.
constexpr int kMfmaMaxCols = 128;

// Chunking and work-buffer sizes of apply_forward_mfma_block.
struct MfmaLayout {
    int tg, nb, ncol;
    int64_t chG, chF;
    int ncG, ncF;
    int64_t fstride, ldqG, ldqF;
    size_t part, qG, qF;
};
MfmaLayout mfma_layout(const vsie_problem *p, int nf, int nrhs) {
    const int64_t n = p->m.n;
    MfmaLayout L;
    L.tg = p->tune.mfma_tg;
    L.nb = p->tune.mfma_nb;
    const int cbw = 16 * L.nb;
    L.ncol = (nrhs + cbw - 1) / cbw * cbw;
    const int grid = mfma_grid(L.tg, L.nb);
    const int64_t want = static_cast<int64_t>(grid) * (kBlock / 64) * p->tune.items_per_wave;
    const int64_t tiles = (n + 16 * L.tg - 1) / (16 * L.tg);
    const int64_t items_per_chunk = static_cast<int64_t>(nf) * (L.ncol / cbw) * tiles;
    auto chunking = [&](int64_t ns, int64_t &chunk, int &nc) {
        if (ns <= 0) {
            chunk = 4;
            nc = 0;
            return;
        }
        int64_t c = (want + items_per_chunk - 1) / items_per_chunk;
        c = std::max<int64_t>(1, std::min<int64_t>(c, std::max<int64_t>(1, ns / 512)));
        const int64_t cap = p->tune.mfma_chunk_max;
        if (cap > 0) c = std::max<int64_t>(c, (ns + cap - 1) / cap);
        chunk = ((ns + c - 1) / c + 3) / 4 * 4;
        nc = static_cast<int>((ns + chunk - 1) / chunk);
    };
    chunking(p->G.count, L.chG, L.ncG);
    chunking(p->F.count, L.chF, L.ncF);
    L.fstride = static_cast<int64_t>(L.ncG + L.ncF) * nrhs * n;
    L.part = sizeof(double2) * static_cast<size_t>(std::max<int64_t>(1, L.fstride * nf));
    L.ldqG = (p->G.count + kMfmaPad) * L.ncol;
    L.ldqF = (p->F.count + kMfmaPad) * L.ncol;
    L.qG = sizeof(float2) * static_cast<size_t>(L.ldqG * nf);
    L.qF = sizeof(float2) * static_cast<size_t>(L.ldqF * nf);
    return L;
}

void apply_forward_mfma_block(vsie_problem *p, int f0, int nf, int nrhs, const double2 *x, int64_t ldx,
                              int64_t xfs, double2 *y, int64_t ldy, int64_t yfs, hipStream_t s) {
    const int64_t n = p->m.n;
    const MfmaLayout L = mfma_layout(p, nf, nrhs);
    const int tg = L.tg, nb = L.nb, ncol = L.ncol;
    const int64_t chG = L.chG, chF = L.chF;
    const int ncG = L.ncG, ncF = L.ncF;
    const int parts = ncG + ncF;
    const int64_t fstride = L.fstride;
    double2 *part = static_cast<double2 *>(p->partial.get(L.part));
    const int64_t ldqG = L.ldqG, ldqF = L.ldqF;
    float2 *qG = static_cast<float2 *>(p->chargeG.get(L.qG));
    float2 *qF = static_cast<float2 *>(p->chargeF.get(L.qF));
    const double *kf = p->d_k0 + f0;
    if (ncG > 0) {
        launch_pack_mfma(kClassG, p->G, p->m.sp + static_cast<int64_t>(f0) * n, n, nf, nrhs, ncol, x, ldx, xfs,
                         qG, ldqG, s);
        MfmaJob J{kClassG, n, p->m.px, p->m.py, p->m.pz, p->G.count, p->G.pk, nullptr, qG, ldqG, ncol, nrhs,
                  kf, nf, chG, ncG, part, fstride, 0, tg, nb, 0, p->tune.mfma_3m != 0};
        launch_mfma_forward(J, s, &p->prof);
    }
    if (ncF > 0) {
        launch_pack_mfma(kClassF, p->F, nullptr, n, nf, nrhs, ncol, x, ldx, xfs, qF, ldqF, s);
        MfmaJob J{kClassF, n, p->m.px, p->m.py, p->m.pz, p->F.count, p->F.pk, p->F.pv, qF, ldqF, ncol, nrhs,
                  kf, nf, chF, ncF, part, fstride, ncG, tg, nb, 0, p->tune.mfma_3m != 0};
        launch_mfma_forward(J, s, &p->prof);
    }
    for (int t = 0; t < nf; ++t)
        launch_reduce_partials(n, nrhs, parts, part + t * fstride, p->m.diag + static_cast<int64_t>(f0 + t) * n,
                               false, x + t * xfs, ldx, y + t * yfs, ldy, nullptr, s);
}

void plan_forward_mfma(vsie_problem *p, int nf, int nrhs, WsPlan &pl) {
    for (int r0 = 0; r0 < nrhs; r0 += kMfmaMaxCols) {
        const MfmaLayout L = mfma_layout(p, nf, std::min(kMfmaMaxCols, nrhs - r0));
        pl.need(p->partial, L.part);
        pl.need(p->chargeG, L.qG);
        pl.need(p->chargeF, L.qF);
    }
}

void apply_forward_mfma(vsie_problem *p, int f0, int nf, int nrhs, const double2 *x, int64_t ldx, int64_t xfs,
                        double2 *y, int64_t ldy, int64_t yfs, hipStream_t s) {
    for (int r0 = 0; r0 < nrhs; r0 += kMfmaMaxCols) {
        const int blk = std::min(kMfmaMaxCols, nrhs - r0);
        apply_forward_mfma_block(p, f0, nf, blk, x + static_cast<int64_t>(r0) * ldx, ldx, xfs,
                                 y + static_cast<int64_t>(r0) * ldy, ldy, yfs, s);
    }
}

bool use_mfma(const vsie_problem *p, vsie_precision prec, int nrhs) {
    return prec == VSIE_FP32 && p->tune.mfma_min_rhs > 0 && nrhs >= p->tune.mfma_min_rhs;
}

bool use_mfma64(const vsie_problem *p, vsie_precision prec, int nrhs) {
    return prec == VSIE_FP64 && p->tune.mfma64_min_rhs > 0 && nrhs >= p->tune.mfma64_min_rhs;
}

// FP64 forward products on the FP64 matrix cores for the nf frequencies f0 ..
// (layout as apply_forward_mfma): 16, 32 or 64 columns per kernel evaluation
// by the width of the block, at most kMfmaMaxCols columns per pass.
struct Mfma64Layout {
    int nb, ncol;
    int64_t chG, chF;
    int ncG, ncF;
    int64_t fstride, ldqG, ldqF;
    size_t part, qG, qF;
};
Mfma64Layout mfma64_layout(const vsie_problem *p, int nf, int nrhs) {
    const int64_t n = p->m.n;
    Mfma64Layout L;
    L.nb = nrhs <= 16 ? 1 : (nrhs <= 32 ? 2 : 4);
    const int cbw = 16 * L.nb;
    L.ncol = (nrhs + cbw - 1) / cbw * cbw;
    const int64_t want = static_cast<int64_t>(mfma_grid(2, 1)) * (kBlock / 64) * p->tune.items_per_wave;
    // target tiles of 16 mfma64_groups points
    auto chunking = [&](int64_t ns, int64_t tile_pts, int64_t &chunk, int &nc) {
        if (ns <= 0) {
            chunk = 4;
            nc = 0;
            return;
        }
        const int64_t items_per_chunk = static_cast<int64_t>(nf) * (L.ncol / cbw) * ((n + tile_pts - 1) / tile_pts);
        int64_t c = (want + items_per_chunk - 1) / items_per_chunk;
        c = std::max<int64_t>(1, std::min<int64_t>(c, std::max<int64_t>(1, ns / 512)));
        const int64_t cap = p->tune.mfma_chunk_max;
        if (cap > 0) c = std::max<int64_t>(c, (ns + cap - 1) / cap);
        chunk = ((ns + c - 1) / c + 3) / 4 * 4;
        nc = static_cast<int>((ns + chunk - 1) / chunk);
    };
    chunking(p->G.count, 16 * mfma64_groups(kClassG, L.nb), L.chG, L.ncG);
    chunking(p->F.count, 16 * mfma64_groups(kClassF, L.nb), L.chF, L.ncF);
    L.fstride = static_cast<int64_t>(L.ncG + L.ncF) * nrhs * n;
    L.part = sizeof(double2) * static_cast<size_t>(std::max<int64_t>(1, L.fstride * nf));
    L.ldqG = (p->G.count + kMfmaPad) * L.ncol;
    L.ldqF = (p->F.count + kMfmaPad) * L.ncol;
    L.qG = sizeof(double2) * static_cast<size_t>(L.ldqG * nf);
    L.qF = sizeof(double2) * static_cast<size_t>(L.ldqF * nf);
    return L;
}

void apply_forward_mfma64_block(vsie_problem *p, int f0, int nf, int nrhs, const double2 *x, int64_t ldx,
                                int64_t xfs, double2 *y, int64_t ldy, int64_t yfs, hipStream_t s) {
    const int64_t n = p->m.n;
    const Mfma64Layout L = mfma64_layout(p, nf, nrhs);
    const int parts = L.ncG + L.ncF;
    double2 *part = static_cast<double2 *>(p->partial.get(L.part));
    double2 *qG = static_cast<double2 *>(p->chargeG.get(L.qG));
    double2 *qF = static_cast<double2 *>(p->chargeF.get(L.qF));
    const double *kf = p->d_k0 + f0;
    const bool m3 = p->tune.mfma_3m != 0;
    if (L.ncG > 0) {
        launch_pack_mfma64(kClassG, p->G, p->m.sp + static_cast<int64_t>(f0) * n, n, nf, nrhs, L.ncol, x, ldx, xfs,
                           qG, L.ldqG, s);
        Mfma64Job J{kClassG, n, p->m.px, p->m.py, p->m.pz, p->G.count, p->G.pk, nullptr, qG, L.ldqG, L.ncol, nrhs,
                    kf, nf, L.chG, L.ncG, part, L.fstride, 0, L.nb, m3};
        launch_mfma64_forward(J, s, &p->prof);
    }
    if (L.ncF > 0) {
        launch_pack_mfma64(kClassF, p->F, nullptr, n, nf, nrhs, L.ncol, x, ldx, xfs, qF, L.ldqF, s);
        Mfma64Job J{kClassF, n, p->m.px, p->m.py, p->m.pz, p->F.count, p->F.pk, p->F.pv, qF, L.ldqF, L.ncol, nrhs,
                    kf, nf, L.chF, L.ncF, part, L.fstride, L.ncG, L.nb, m3};
        launch_mfma64_forward(J, s, &p->prof);
    }
    for (int t = 0; t < nf; ++t)
        launch_reduce_partials(n, nrhs, parts, part + t * L.fstride, p->m.diag + static_cast<int64_t>(f0 + t) * n,
                               false, x + t * xfs, ldx, y + t * yfs, ldy, nullptr, s);
}

void apply_forward_mfma64(vsie_problem *p, int f0, int nf, int nrhs, const double2 *x, int64_t ldx, int64_t xfs,
                          double2 *y, int64_t ldy, int64_t yfs, hipStream_t s) {
    for (int r0 = 0; r0 < nrhs; r0 += kMfmaMaxCols) {
        const int blk = std::min(kMfmaMaxCols, nrhs - r0);
        apply_forward_mfma64_block(p, f0, nf, blk, x + static_cast<int64_t>(r0) * ldx, ldx, xfs,
                                   y + static_cast<int64_t>(r0) * ldy, ldy, yfs, s);
    }
}

void plan_forward_mfma64(vsie_problem *p, int nf, int nrhs, WsPlan &pl) {
    for (int r0 = 0; r0 < nrhs; r0 += kMfmaMaxCols) {
        const Mfma64Layout L = mfma64_layout(p, nf, std::min(kMfmaMaxCols, nrhs - r0));
        pl.need(p->partial, L.part);
        pl.need(p->chargeG, L.qG);
        pl.need(p->chargeF, L.qF);
    }
}

void check_tuning(const vsie_tuning &t) {
    require(t.mfma_min_rhs >= 0, "mfma_min_rhs must be >= 0");
    require((t.mfma_tg == 2 || t.mfma_tg == 4) && (t.mfma_nb == 1 || t.mfma_nb == 2) &&
                mfma_variant_ok(t.mfma_tg, t.mfma_nb),
            "unsupported (mfma_tg, mfma_nb)");
    require(t.items_per_wave >= 1 && t.items_per_wave <= 4096, "items_per_wave must be in [1, 4096]");
    require(t.vec_target_waves >= 1024 && t.vec_target_waves <= (int64_t(1) << 24),
            "vec_target_waves must be in [1024, 2^24]");
    require(t.graph == 0 || t.graph == 1, "graph must be 0 or 1");
    require(t.sym_groups == 0 || (t.sym_groups > 1 && sym_groups_ok(t.sym_groups)), "sym_groups must be 0, 2, 4 or 8");
    require(t.cell_face == 0 || t.cell_face == 1, "cell_face must be 0 or 1");
    require(t.mfma_3m == 0 || t.mfma_3m == 1, "mfma_3m must be 0 or 1");
    require(t.mfma64_min_rhs >= 0, "mfma64_min_rhs must be >= 0");
    require(t.mfma_chunk_max == 0 || t.mfma_chunk_max >= 1024, "mfma_chunk_max must be 0 or >= 1024");
}

// The work buffers of apply_op (same dispatch).
void plan_op(vsie_problem *p, int f, vsie_precision prec, bool adjoint, int nrhs, WsPlan &pl) {
    if (prec == VSIE_FP32 && p->dense[f].A) plan_dense(p, nrhs, pl);
    else if (adjoint) plan_adjoint(p, prec, nrhs, pl);
    else if (use_mfma(p, prec, nrhs)) plan_forward_mfma(p, 1, nrhs, pl);
    else if (use_mfma64(p, prec, nrhs)) plan_forward_mfma64(p, 1, nrhs, pl);
    else plan_forward(p, prec, nrhs, pl);
}

// The work buffers of vsie_matvec_multi (same dispatch).
void plan_multi(vsie_problem *p, int f0, int nf, vsie_precision prec, int nrhs, WsPlan &pl) {
    bool dense = false;
    for (int t = 0; t < nf; ++t) dense = dense || p->dense[f0 + t].A != nullptr;
    if (use_mfma(p, prec, nrhs) && !dense) {
        plan_forward_mfma(p, nf, nrhs, pl);
        return;
    }
    if (use_mfma64(p, prec, nrhs)) {
        plan_forward_mfma64(p, nf, nrhs, pl);
        return;
    }
    for (int t = 0; t < nf; ++t) plan_op(p, f0 + t, prec, false, nrhs, pl);
}

void apply_op(vsie_problem *p, int f, vsie_precision prec, bool adjoint, int nrhs,
              const double2 *x, int64_t ldx, double2 *y, int64_t ldy, hipStream_t s) {
    if (prec == VSIE_FP32 && p->dense[f].A) apply_dense(p, f, adjoint, nrhs, x, ldx, y, ldy, s);
    else if (adjoint) apply_adjoint(p, f, prec, nrhs, x, ldx, y, ldy, s);
    else if (use_mfma(p, prec, nrhs)) apply_forward_mfma(p, f, 1, nrhs, x, ldx, 0, y, ldy, 0, s);
    else if (use_mfma64(p, prec, nrhs)) apply_forward_mfma64(p, f, 1, nrhs, x, ldx, 0, y, ldy, 0, s);
    else apply_forward(p, f, prec, nrhs, x, ldx, y, ldy, s);
}

// apply_op through a hipGraph of its launches, for the fixed work buffers the
// solver applies the operator to every iteration.  The first call with a key
// runs eagerly (which sizes every work buffer and gives this call's product)
// and then captures the same launches; later calls launch the graph.  Every
// path launches kernels only (no memset or copy nodes).  Profiled products
// stay eager.
constexpr size_t kMaxGraphs = 16;

void apply_op_graph(vsie_problem *p, int f, vsie_precision prec, bool adjoint, int nrhs,
                    const double2 *x, int64_t ldx, double2 *y, int64_t ldy, hipStream_t s) {
    if (!p->tune.graph || p->prof.on) {
        apply_op(p, f, prec, adjoint, nrhs, x, ldx, y, ldy, s);
        return;
    }
    const uint64_t ep = g_graph_epoch.load();
    for (auto &q : p->graphs)
        if (q.epoch != ep) {
            p->clear_graphs();
            break;
        }
    for (auto &q : p->graphs)
        if (q.f == f && q.prec == prec && q.adjoint == adjoint && q.nrhs == nrhs && q.x == x && q.ldx == ldx &&
            q.y == y && q.ldy == ldy) {
            VSIE_HIP(hipGraphLaunch(q.e, s));
            return;
        }
    apply_op(p, f, prec, adjoint, nrhs, x, ldx, y, ldy, s);
    if (g_graph_epoch.load() != ep) return;  // buffers were resized on the way: capture next time
    if (p->graphs.size() >= kMaxGraphs) p->clear_graphs();
    // the caller's stream may be the legacy null stream, which cannot be captured
    if (!p->capture_stream) VSIE_HIP(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = p->capture_stream;
    VSIE_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
        apply_op(p, f, prec, adjoint, nrhs, x, ldx, y, ldy, cs);
    } catch (...) {
        (void)hipStreamEndCapture(cs, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    VSIE_HIP(hipStreamEndCapture(cs, &g));
    hipGraphExec_t e = nullptr;
    const hipError_t ie = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        check_hip(ie, "hipGraphInstantiate");
    }
    p->graphs.push_back(vsie_problem::OpGraph{f, static_cast<int>(prec), nrhs, adjoint, x, ldx, y, ldy, ep, g, e});
}

// ---------------------------------------------------------------------------
// GMRES over a batch of right-hand sides
//
// Every right-hand side runs its own GMRES(m); the batch advances in lockstep
// so that each iteration applies the operator to all live right-hand sides in
// one multi-RHS pair launch.  The Krylov basis of rhs r keeps vector j at
// V + (j R + r) n.  Arnoldi uses classical Gram-Schmidt twice (CGS2); the
// Hessenberg columns come to the host once per iteration for the Givens
// rotations and the convergence test of each rhs.

struct SolveCounters {
    std::vector<int> it, mv64, mv32, outer;
    explicit SolveCounters(int R) : it(R, 0), mv64(R, 0), mv32(R, 0), outer(R, 0) {}
};

// host copy of a small device array, after the stream has drained
template <typename T>
void to_host(std::vector<T> &h, const T *d, size_t count, hipStream_t s) {
    h.resize(count);
    if (count) VSIE_HIP(hipMemcpyAsync(h.data(), d, sizeof(T) * count, hipMemcpyDeviceToHost, s));
    VSIE_HIP(hipStreamSynchronize(s));
}

template <typename T>
void to_device(T *d, const std::vector<T> &h, hipStream_t s) {
    if (h.empty()) return;
    VSIE_HIP(hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s));
    VSIE_HIP(hipStreamSynchronize(s));  // h may change right after
}

// Cap on the two Krylov bases together: vsie_solve_opts.krylov_gib GiB, by
// default 96 GiB of the 288 GB (room for c2's 108.5 GB assembled operator).
constexpr int64_t kKrylovDefaultGiB = 96;
int64_t krylov_bytes(const vsie_solve_opts &o) {
    return (o.krylov_gib > 0 ? static_cast<int64_t>(o.krylov_gib) : kKrylovDefaultGiB) << 30;
}

int norm_chunks(int64_t n) { return static_cast<int>(std::min<int64_t>(256, std::max<int64_t>(1, n / 2048))); }

// 2-norms of nslots contiguous columns of length n
std::vector<double> column_norms(vsie_problem *p, const double2 *W, int nslots, hipStream_t s) {
    const int64_t n = p->m.n;
    const int nch = norm_chunks(n);
    double *part = static_cast<double *>(p->npart.get(sizeof(double) * nch * std::max(1, nslots)));
    double *out = static_cast<double *>(p->nrm.get(sizeof(double) * std::max(1, nslots)));
    bblas_norm(n, nslots, W, part, nch, out, s);
    std::vector<double> h;
    to_host(h, out, nslots, s);
    return h;
}

using cd = std::complex<double>;

// run fn(i) for i in [0, count) on up to 16 host threads; `work` is the
// whole loop's approximate flop count.  Starting and joining the threads
// costs a few hundred microseconds, so loops below kThreadMinWork (about that
// much serial work) run on the calling thread.
constexpr double kThreadMinWork = 1e6;

template <typename Fn>
void parallel_for(int count, double work, Fn fn) {
    const int nt = work < kThreadMinWork
                       ? 1
                       : std::max(1, std::min<int>({count, 16, static_cast<int>(std::thread::hardware_concurrency())}));
    if (nt <= 1) {
        for (int i = 0; i < count; ++i) fn(i);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int i = t; i < count; i += nt) fn(i);
        });
    for (auto &x : th) x.join();
}


// Y <- R^{-1} Y for an upper triangular R (k x k, column-major, leading
// dimension ld) and nc right-hand sides (Y column-major k x nc, ldy = k); a
// zero pivot gives a zero component.  Columns go in blocks of kTriBlock to
// the host threads; each block is solved column-oriented (y_i /= R_ii, then
// the rows above lose R(0:i, i) y_i), so R is read one contiguous column at a
// time, once per block.  (The row-oriented form reads R(i, i+1:k) at stride
// ld: one cache miss per entry, about 40 times slower at k = 2688.)
constexpr int kTriBlock = 8;

// col(i) points at column i of R (entries 0..i contiguous)
template <typename Col>
void tri_solve_upper_cols_by(Col col, int64_t k, int nc, cd *Y) {
    if (k <= 0 || nc <= 0) return;
    const int nblk = (nc + kTriBlock - 1) / kTriBlock;
    parallel_for(nblk, 4.0 * static_cast<double>(k) * k * nc, [&](int b) {
        const int c0 = b * kTriBlock, nb = std::min(kTriBlock, nc - c0);
        // block rows i: kTriBlock interleaved (re, im) pairs
        std::vector<double> Yb(static_cast<size_t>(k) * 2 * kTriBlock, 0.0);
        for (int c = 0; c < nb; ++c)
            for (int64_t i = 0; i < k; ++i) {
                const cd v = Y[(c0 + c) * k + i];
                Yb[(i * kTriBlock + c) * 2] = v.real();
                Yb[(i * kTriBlock + c) * 2 + 1] = v.imag();
            }
        for (int64_t i = k - 1; i >= 0; --i) {
            const cd *Rc = col(i);
            const cd d = Rc[i];
            double *yi = &Yb[i * 2 * kTriBlock];
            for (int c = 0; c < kTriBlock; ++c) {
                const cd v = d == 0.0 ? cd(0.0) : cd(yi[2 * c], yi[2 * c + 1]) / d;
                yi[2 * c] = v.real();
                yi[2 * c + 1] = v.imag();
            }
            const double *Ri = reinterpret_cast<const double *>(Rc);
            for (int64_t t = 0; t < i; ++t) {
                const double rr = Ri[2 * t], ri = Ri[2 * t + 1];
                double *yt = &Yb[t * 2 * kTriBlock];
                for (int c = 0; c < kTriBlock; ++c) {
                    const double ar = yi[2 * c], ai = yi[2 * c + 1];
                    yt[2 * c] -= rr * ar - ri * ai;
                    yt[2 * c + 1] -= rr * ai + ri * ar;
                }
            }
        }
        for (int c = 0; c < nb; ++c)
            for (int64_t i = 0; i < k; ++i)
                Y[(c0 + c) * k + i] = cd(Yb[(i * kTriBlock + c) * 2], Yb[(i * kTriBlock + c) * 2 + 1]);
    });
}

// R column-major with leading dimension ld
void tri_solve_upper_cols(const cd *R, int64_t ld, int64_t k, int nc, cd *Y) {
    tri_solve_upper_cols_by([&](int64_t i) { return R + i * ld; }, k, nc, Y);
}

// Upper triangle stored by columns, packed: column c holds its c + 1
// entries at offset c (c + 1) / 2.
inline size_t packed_col(int64_t c) { return static_cast<size_t>(c) * (c + 1) / 2; }

// The Krylov space of a finished cycle, kept to deflate later cycles (GCRO):
// the cycle's Arnoldi relation A V_k = V_{k+1} Hbar with Hbar = Q R by the
// cycle's own Givens rotations gives C = V_{k+1} Q (orthonormal) and
// U = V_k R^{-1} with A U = C.  Later cycles solve with (I - C C^H) A, start
// from the correction U C^H r, and correct their result by -U B y.
struct RecycleRhs {
    int k = 0;
    std::vector<cd> cs, sn;  // rotations 0..k-1
    std::vector<cd> Rm;      // k x k upper triangle, column-major
};
struct Recycle {
    const double2 *V = nullptr;  // basis buffer of the recycled cycle (layout of gmres_cycle)
    std::vector<RecycleRhs> rhs;  // indexed by right-hand side
};

// t <- G_{k-1} ... G_0 t for t of length k + 1 (G_j = [[conj c, conj s], [-s, c]] on rows j, j+1)
void rot_fwd(const RecycleRhs &q, std::vector<cd> &t) {
    for (int j = 0; j < q.k; ++j) {
        const cd a = t[j], b = t[j + 1];
        t[j] = std::conj(q.cs[j]) * a + std::conj(q.sn[j]) * b;
        t[j + 1] = -q.sn[j] * a + q.cs[j] * b;
    }
}
// v <- G_0^H ... G_{k-1}^H v
void rot_bwd(const RecycleRhs &q, std::vector<cd> &v) {
    for (int j = q.k - 1; j >= 0; --j) {
        const cd a = v[j], b = v[j + 1];
        v[j] = q.cs[j] * a - std::conj(q.sn[j]) * b;
        v[j + 1] = q.sn[j] * a + std::conj(q.cs[j]) * b;
    }
}
// R y = c
std::vector<cd> r_solve(const RecycleRhs &q, const std::vector<cd> &c) {
    std::vector<cd> y(q.k);
    for (int i = q.k - 1; i >= 0; --i) {
        cd acc = c[i];
        for (int j = i + 1; j < q.k; ++j) acc -= q.Rm[static_cast<size_t>(j) * q.k + i] * y[j];
        y[i] = acc / q.Rm[static_cast<size_t>(i) * q.k + i];
    }
    return y;
}

// One GMRES cycle for the right-hand sides rhs[0..ns) (slot order), with
// residual block Rres (ns x n, norms rn; overwritten when `use` projects it)
// and per-slot stopping tolerances; adds the corrections to x.  The basis is
// written to Vb.  `save` receives this cycle's space for later deflation;
// `use` deflates this cycle with an earlier one.  Returns the iterations done.
int gmres_cycle(vsie_problem *p, int f, vsie_precision prec, bool adjoint, int R,
                const std::vector<int32_t> &rhs, double2 *Rres, const std::vector<double> &rn,
                const std::vector<double> &ctol, int m, int iter_cap, double2 *x, int64_t ldx,
                SolveCounters &cnt, hipStream_t s, double2 *Vb, Recycle *save, const Recycle *use,
                double relax) {
    const int64_t n = p->m.n;
    const int ns = static_cast<int>(rhs.size());
    const int hs = m + 2;  // stride of per-slot coefficient vectors
    int kmax = 0;          // largest recycled dimension in this batch
    if (use)
        for (int r : rhs) kmax = std::max(kmax, use->rhs[r].k);
    const int cs_ = std::max(hs, kmax + 2);
    double2 *V = Vb;
    double2 *W = static_cast<double2 *>(p->w.get(sizeof(double2) * static_cast<size_t>(n) * ns));
    double2 *X = static_cast<double2 *>(p->ax.get(sizeof(double2) * static_cast<size_t>(n) * ns));
    // both Gram-Schmidt passes' coefficients and the new norms in one block, so
    // that one copy brings an iteration's Hessenberg column to the host
    const size_t hcol_bytes = sizeof(double2) * 2 * static_cast<size_t>(hs) * ns + sizeof(double) * ns;
    double2 *h1 = static_cast<double2 *>(p->h1.get(hcol_bytes));
    double2 *h2 = h1 + static_cast<size_t>(hs) * ns;
    double *hn = reinterpret_cast<double *>(h2 + static_cast<size_t>(hs) * ns);
    double2 *tc = static_cast<double2 *>(p->tc.get(sizeof(double2) * static_cast<size_t>(cs_) * ns));
    const int nch = norm_chunks(n);
    double2 *dpart = static_cast<double2 *>(
        p->dpart.get(sizeof(double2) * static_cast<size_t>(nch) * std::max(m + 1, kmax + 1) * ns));
    double *npart = static_cast<double *>(p->npart.get(sizeof(double) * nch * ns));
    double *nrm = static_cast<double *>(p->nrm.get(sizeof(double) * ns));
    int32_t *act = static_cast<int32_t *>(p->act.get(sizeof(int32_t) * ns));
    int32_t *live_d = static_cast<int32_t *>(p->live.get(sizeof(int32_t) * ns));
    int32_t *kc_d = static_cast<int32_t *>(p->kc.get(sizeof(int32_t) * ns));
    // coefficient uploads use strides up to cs_ (>= max(m + 1, kmax + 1))
    double2 *yv = static_cast<double2 *>(p->yv.get(sizeof(double2) * static_cast<size_t>(cs_) * ns));
    int32_t *kd_d = static_cast<int32_t *>(p->kd.get(sizeof(int32_t) * ns));

    to_device(act, rhs, s);
    std::vector<double> beta0(rn);
    std::vector<int32_t> kcnt(ns, 0);
    if (use && kmax > 0) {
        // project the residuals: x += U C^H r, r -= C C^H r
        for (int sl = 0; sl < ns; ++sl) {
            const int kr = use->rhs[rhs[sl]].k;
            kcnt[sl] = kr > 0 ? kr + 1 : 0;
        }
        to_device(kc_d, kcnt, s);
        bblas_dots(n, kmax + 1, R, ns, act, use->V, Rres, dpart, nch, tc, cs_, s);
        std::vector<double2> th;
        to_host(th, tc, static_cast<size_t>(cs_) * ns, s);
        std::vector<double2> sv(static_cast<size_t>(cs_) * ns, make_double2(0, 0)), uv(sv);
        std::vector<int32_t> ku(ns, 0);
        for (int sl = 0; sl < ns; ++sl) {
            const RecycleRhs &q = use->rhs[rhs[sl]];
            if (q.k == 0) continue;
            std::vector<cd> t(q.k + 1);
            for (int j = 0; j <= q.k; ++j) t[j] = cd(th[sl * cs_ + j].x, th[sl * cs_ + j].y);
            rot_fwd(q, t);
            std::vector<cd> c(t.begin(), t.begin() + q.k);
            const std::vector<cd> y0 = r_solve(q, c);
            std::vector<cd> v(q.k + 1, 0.0);
            for (int j = 0; j < q.k; ++j) v[j] = c[j];
            rot_bwd(q, v);
            for (int j = 0; j <= q.k; ++j) sv[sl * cs_ + j] = make_double2(v[j].real(), v[j].imag());
            for (int j = 0; j < q.k; ++j) uv[sl * cs_ + j] = make_double2(y0[j].real(), y0[j].imag());
            ku[sl] = q.k;
        }
        to_device(tc, sv, s);
        bblas_gemv_sub(n, kmax + 1, R, ns, act, use->V, tc, cs_, Rres, s, kc_d);
        to_device(yv, uv, s);
        to_device(kd_d, ku, s);
        bblas_update(n, R, ns, act, kd_d, use->V, yv, cs_, x, ldx, s);
        const std::vector<double> b2 = column_norms(p, Rres, ns, s);
        beta0 = b2;
    }
    // Deflation inside the cycle, W -= C C^H W with C = V1 Q (Q: the first k
    // columns of the recycled cycle's rotations), runs on the device: per slot
    // P = Q Q^H ((k+1) x (k+1)) turns the projections t = V1^H W into the
    // update coefficients, and Q^H t (k entries) is summed into B (column j
    // for step j: B = C^H A V, needed for the final correction).  P and Q^H
    // are built once per cycle by rotating unit vectors.
    const size_t pm = static_cast<size_t>(cs_) * cs_;
    const int64_t bstride = static_cast<int64_t>(m) * kmax;
    double2 *Pd = nullptr, *Md = nullptr, *Bd = nullptr;
    int32_t *kcs_d = nullptr, *lslot_d = nullptr;
    if (use && kmax > 0) {
        std::vector<double2> Ph(pm * ns, make_double2(0.0, 0.0)), Mh(pm * ns, make_double2(0.0, 0.0));
        parallel_for(ns, 24.0 * ns * (kmax + 1) * kmax, [&](int sl) {
            const RecycleRhs &q = use->rhs[rhs[sl]];
            if (q.k == 0) return;
            std::vector<cd> t(q.k + 1), v(q.k + 1);
            for (int j = 0; j <= q.k; ++j) {
                std::fill(t.begin(), t.end(), cd(0.0));
                t[j] = 1.0;
                rot_fwd(q, t);
                for (int i = 0; i < q.k; ++i) {
                    Mh[sl * pm + static_cast<size_t>(j) * cs_ + i] = make_double2(t[i].real(), t[i].imag());
                    v[i] = t[i];
                }
                v[q.k] = 0.0;
                rot_bwd(q, v);
                for (int i = 0; i <= q.k; ++i)
                    Ph[sl * pm + static_cast<size_t>(j) * cs_ + i] = make_double2(v[i].real(), v[i].imag());
            }
        });
        Pd = static_cast<double2 *>(p->defP.get(sizeof(double2) * pm * ns));
        Md = static_cast<double2 *>(p->defM.get(sizeof(double2) * pm * ns));
        Bd = static_cast<double2 *>(p->defB.get(sizeof(double2) * static_cast<size_t>(bstride) * ns));
        kcs_d = static_cast<int32_t *>(p->defk.get(sizeof(int32_t) * ns));
        lslot_d = static_cast<int32_t *>(p->lslot.get(sizeof(int32_t) * ns));
        to_device(Pd, Ph, s);
        to_device(Md, Mh, s);
        to_device(kcs_d, kcnt, s);
        blas_zero(bstride * ns, Bd, s);
    }
    // v0 = r / |r| (a zero projected residual gives a zero vector and stops at once)
    to_device(nrm, beta0, s);
    bblas_scale_into_basis(n, 0, R, ns, act, Rres, nrm, V, s);

    std::vector<std::vector<cd>> H(ns, std::vector<cd>(static_cast<size_t>(m + 1) * m, 0.0));
    std::vector<std::vector<cd>> cs(ns, std::vector<cd>(m)), sn(ns, std::vector<cd>(m)),
        g(ns, std::vector<cd>(m + 1, 0.0));
    std::vector<int> kdone(ns, 0);
    std::vector<char> done(ns, 0);
    for (int sl = 0; sl < ns; ++sl) {
        g[sl][0] = beta0[sl];
        if (beta0[sl] <= ctol[sl] * rn[sl]) done[sl] = 1;  // the projection already solved it
    }
    std::vector<int32_t> live_prev;  // live list last uploaded to live_d
    std::vector<double> hbeta;
    int total = 0;
    for (int k = 0; k < m; ++k) {
        std::vector<int32_t> live_rhs, live_slot, live_kc;
        for (int sl = 0; sl < ns; ++sl)
            if (!done[sl] && cnt.it[rhs[sl]] < iter_cap) {
                live_rhs.push_back(rhs[sl]);
                live_slot.push_back(sl);
                live_kc.push_back(kcnt[sl]);
            }
        const int nl = static_cast<int>(live_rhs.size());
        if (nl == 0) break;
        if (live_rhs != live_prev) {
            to_device(live_d, live_rhs, s);
            if (use && kmax > 0) {
                std::vector<int32_t> ls(live_slot.begin(), live_slot.end());
                to_device(lslot_d, ls, s);
                to_device(kc_d, live_kc, s);
            }
            live_prev = live_rhs;
        }
        // W = A v_k for the live right-hand sides; with relaxed products the FP64
        // operator while any live residual estimate is above its switch point
        vsie_precision iprec = prec;
        if (prec == VSIE_FP32 && relax > 0)
            for (int l = 0; l < nl; ++l) {
                const int sl = live_slot[l];
                if (std::abs(g[sl][k]) > ctol[sl] * rn[sl] / relax) iprec = VSIE_FP64;
            }
        bblas_gather(n, nl, live_d, V + static_cast<int64_t>(k) * R * n, n, X, s);
        apply_op_graph(p, f, iprec, adjoint, nl, X, n, W, n, s);
        for (int r : live_rhs) (iprec == VSIE_FP64 ? cnt.mv64 : cnt.mv32)[r]++;
        for (int pass = 0; pass < 2; ++pass) {
            double2 *h = pass == 0 ? h1 : h2;
            if (use && kmax > 0) {
                // deflation: t = V1^H W, W -= V1 (P t), B column k += Q^H t
                bblas_dots(n, kmax + 1, R, nl, live_d, use->V, W, dpart, nch, tc, cs_, s);
                bblas_deflate_coef(nl, lslot_d, kcs_d, cs_, Pd, Md, tc, yv, Bd, k, kmax, bstride, s);
                bblas_gemv_sub(n, kmax + 1, R, nl, live_d, use->V, yv, cs_, W, s, kc_d);
            }
            if (bblas_fused_ok(k + 1)) {
                bblas_dots_partial(n, k + 1, R, nl, live_d, V, W, dpart, nch, s);
                bblas_gemv_sub_partial(n, k + 1, R, nl, live_d, V, dpart, nch, h, hs, W, s);
            } else {
                bblas_dots(n, k + 1, R, nl, live_d, V, W, dpart, nch, h, hs, s);
                bblas_gemv_sub(n, k + 1, R, nl, live_d, V, h, hs, W, s);
            }
        }
        bblas_norm_partial(n, nl, W, npart, nch, s);
        bblas_norm_scale(n, k + 1, R, nl, live_d, W, npart, nch, hn, V, s);
        // both Gram-Schmidt passes' coefficients and the new norm, in one copy
        double2 *hb1 = static_cast<double2 *>(p->hpin.get(hcol_bytes));
        double2 *hb2 = hb1 + static_cast<size_t>(hs) * ns;
        double *hbeta = reinterpret_cast<double *>(hb2 + static_cast<size_t>(hs) * ns);
        VSIE_HIP(hipMemcpyAsync(hb1, h1, hcol_bytes, hipMemcpyDeviceToHost, s));
        VSIE_HIP(hipStreamSynchronize(s));
        for (int l = 0; l < nl; ++l) {
            const int sl = live_slot[l];
            auto Hat = [&](int i, int j) -> cd & { return H[sl][static_cast<size_t>(j) * (m + 1) + i]; };
            const double beta = hbeta[l];
            if (!std::isfinite(beta)) fail(VSIE_E_NAN, "non-finite value in the Krylov basis");
            for (int j = 0; j <= k; ++j)
                Hat(j, k) = cd(hb1[l * hs + j].x + hb2[l * hs + j].x, hb1[l * hs + j].y + hb2[l * hs + j].y);
            Hat(k + 1, k) = beta;
            // unitary rotations [[conj(c), conj(s)], [-s, c]]
            for (int j = 0; j < k; ++j) {
                const cd a = Hat(j, k), b = Hat(j + 1, k);
                Hat(j, k) = std::conj(cs[sl][j]) * a + std::conj(sn[sl][j]) * b;
                Hat(j + 1, k) = -sn[sl][j] * a + cs[sl][j] * b;
            }
            const cd a = Hat(k, k), b = Hat(k + 1, k);
            const double den = std::hypot(std::abs(a), std::abs(b));
            if (den == 0.0) {  // no new direction: keep the first k columns
                done[sl] = 1;
                continue;
            }
            cs[sl][k] = a / den;
            sn[sl][k] = b / den;
            Hat(k, k) = den;
            Hat(k + 1, k) = 0.0;
            g[sl][k + 1] = -sn[sl][k] * g[sl][k];
            g[sl][k] = std::conj(cs[sl][k]) * g[sl][k];
            cnt.it[rhs[sl]]++;
            ++total;
            kdone[sl] = k + 1;
            if (std::abs(g[sl][k + 1]) <= ctol[sl] * rn[sl] || beta == 0.0) done[sl] = 1;
        }
        if (p->progress && (k + 1) % 25 == 0) {
            double worst = 0.0;
            for (int sl = 0; sl < ns; ++sl) worst = std::max(worst, std::abs(g[sl][kdone[sl]]) / rn[sl]);
            std::fprintf(stderr, "[vsie] GMRES iteration %d: max residual estimate %.3e of the cycle start\n", k + 1,
                         worst);
            std::fflush(stderr);
        }
    }
    // x += V y with H y = g (back substitution per slot), then x -= U (B y)
    std::vector<double2> yh(static_cast<size_t>(std::max(m + 1, kmax + 1)) * ns, make_double2(0.0, 0.0));
    const int ys = std::max(m + 1, kmax + 1);
    std::vector<int32_t> kdh(ns);
    std::vector<std::vector<cd>> ys_all(ns);
    for (int sl = 0; sl < ns; ++sl) {
        const int kk = kdone[sl];
        kdh[sl] = kk;
        auto Hat = [&](int i, int j) -> cd & { return H[sl][static_cast<size_t>(j) * (m + 1) + i]; };
        std::vector<cd> y(kk);
        for (int i = kk - 1; i >= 0; --i) {
            cd acc = g[sl][i];
            for (int j = i + 1; j < kk; ++j) acc -= Hat(i, j) * y[j];
            y[i] = acc / Hat(i, i);
        }
        for (int i = 0; i < kk; ++i) yh[static_cast<size_t>(sl) * ys + i] = make_double2(y[i].real(), y[i].imag());
        ys_all[sl] = y;
    }
    to_device(yv, yh, s);
    to_device(kd_d, kdh, s);
    bblas_update(n, R, ns, act, kd_d, V, yv, ys, x, ldx, s);
    if (use && kmax > 0) {
        std::vector<double2> Bh;
        to_host(Bh, Bd, static_cast<size_t>(bstride) * ns, s);
        std::vector<double2> uh(static_cast<size_t>(ys) * ns, make_double2(0.0, 0.0));
        std::vector<int32_t> ku(ns, 0);
        for (int sl = 0; sl < ns; ++sl) {
            const RecycleRhs &q = use->rhs[rhs[sl]];
            if (q.k == 0 || kdone[sl] == 0) continue;
            std::vector<cd> by(q.k, 0.0);
            for (int j = 0; j < kdone[sl]; ++j)
                for (int i = 0; i < q.k; ++i) {
                    const double2 b = Bh[static_cast<size_t>(sl) * bstride + static_cast<size_t>(j) * kmax + i];
                    by[i] += cd(b.x, b.y) * ys_all[sl][j];
                }
            const std::vector<cd> u = r_solve(q, by);
            for (int i = 0; i < q.k; ++i) uh[static_cast<size_t>(sl) * ys + i] = make_double2(-u[i].real(), -u[i].imag());
            ku[sl] = q.k;
        }
        to_device(yv, uh, s);
        to_device(kd_d, ku, s);
        bblas_update(n, R, ns, act, kd_d, use->V, yv, ys, x, ldx, s);
    }
    if (save) {
        save->V = V;
        save->rhs.assign(R, RecycleRhs{});
        for (int sl = 0; sl < ns; ++sl) {
            RecycleRhs &q = save->rhs[rhs[sl]];
            q.k = kdone[sl];
            q.cs.assign(cs[sl].begin(), cs[sl].begin() + q.k);
            q.sn.assign(sn[sl].begin(), sn[sl].begin() + q.k);
            q.Rm.assign(static_cast<size_t>(q.k) * q.k, 0.0);
            for (int j = 0; j < q.k; ++j)
                for (int i = 0; i <= j; ++i) q.Rm[static_cast<size_t>(j) * q.k + i] = H[sl][static_cast<size_t>(j) * (m + 1) + i];
        }
    }
    VSIE_HIP(hipStreamSynchronize(s));
    return total;
}

// The block Krylov space of a finished block cycle, kept to deflate later
// cycles (block GCRO, as Recycle for one column): the block Arnoldi relation
// A V_k = V_{k+Ra} Hbar with Hbar = Q R by the cycle's Householder reflectors
// gives C = V_{k+Ra} Q(:, 0:k) (orthonormal) and U = V_k R^{-1} with A U = C.
// Kept only while k <= kBlockRecycleMax: Q(:, 0:k) is formed once on the host
// (O(k^2 (Ra + 1)), 16 threads) and held on the device ((k + Ra) k complex),
// and R^{-1} runs on the host at O(k^2) per column once per cycle.
constexpr int64_t kBlockRecycleMax = 4096;

struct BlockRecycle {
    const double2 *V = nullptr;  // basis of the recycled cycle: n x (k + Ra)
    int Ra = 0;                  // block width of that cycle
    int64_t k = 0;               // columns of U and C (0: nothing kept)
    std::vector<cd> R;           // k x k upper triangle, column-major (host)
    // Q E on the device ((k + Ra) x k, column-major): the first k columns of
    // the product of the cycle's Householder reflectors, so that C = V (Q E)
    // and every deflation is three GEMMs on the device
    double2 *Qk = nullptr;
};
int block_cycle(vsie_problem *p, int f, vsie_precision prec, bool adjoint, const std::vector<int32_t> &rhs,
                double2 *Rres, const std::vector<double> &rn, const std::vector<double> &ctol, int m,
                int iter_cap, double2 *x, int64_t ldx, SolveCounters &cnt, hipStream_t s, double2 *V,
                BlockRecycle *save, const BlockRecycle *use, double2 *Bm, double2 *qk);

// Device memory of the block deflation for block widths up to R with
// steps(Ra) block steps per cycle of width Ra: the Q E of one kept space
// (qk bytes), the C^H A V of one cycle (bm bytes) and the per-pass
// coefficients (zt bytes).  A kept space has at most kcap columns.
struct DeflateCaps {
    int64_t kcap = 0, jmax = 0;
    size_t qk = 0, bm = 0, zt = 0;
};
DeflateCaps deflate_caps(int R, const std::function<int(int)> &steps) {
    DeflateCaps c;
    for (int Ra = 1; Ra <= R; ++Ra) c.jmax = std::max<int64_t>(c.jmax, static_cast<int64_t>(Ra) * steps(Ra));
    c.kcap = std::min<int64_t>(c.jmax, kBlockRecycleMax);
    const size_t z = sizeof(double2);
    c.qk = z * static_cast<size_t>(c.kcap + R) * static_cast<size_t>(c.kcap);
    c.bm = z * static_cast<size_t>(c.kcap) * static_cast<size_t>(c.jmax);
    c.zt = z * static_cast<size_t>(c.kcap) * R;
    return c;
}

// Restart length of the independent-GMRES path: as asked, but the two bases
// of all R right-hand sides must fit the Krylov budget.
int gmres_restart(int64_t n, int R, const vsie_solve_opts &o) {
    const int64_t col_bytes = static_cast<int64_t>(sizeof(double2)) * n * R;
    return static_cast<int>(std::max<int64_t>(
        1, std::min<int64_t>(std::max(1, o.restart), krylov_bytes(o) / 2 / col_bytes - 1)));
}

// Block steps per cycle of block GMRES with Ra columns: the requested restart,
// but the host R factor of the block Hessenberg ((m Ra)^2 complex) stays near
// 2 GB and the basis within the budget (half of the Krylov budget each: the
// first cycle's basis is kept to deflate the later ones).
int block_restart(int64_t n, int Ra, const vsie_solve_opts &o) {
    const int64_t mb_host = std::max<int64_t>(1, 11585 / Ra);
    const int64_t mb_dev =
        std::max<int64_t>(1, krylov_bytes(o) / 2 / (static_cast<int64_t>(sizeof(double2)) * n * Ra) - 1);
    return static_cast<int>(std::min<int64_t>({static_cast<int64_t>(std::max(1, o.restart)), mb_host, mb_dev}));
}

// Solve op(A) x_r = b_r for r < R.  FP64: restarted GMRES(m), each restart
// from the true FP64 residual.  FP32: the same loop is iterative refinement --
// residuals with the FP64 operator, corrections from one GMRES cycle with the
// FP32 operator to the inner tolerance.
vsie_status solve_batch(vsie_problem *p, int f, vsie_precision prec, bool adjoint, int R,
                        const double2 *b, int64_t ldb, double2 *x, int64_t ldx,
                        const vsie_solve_opts &o, SolveCounters &cnt, std::vector<double> &relres,
                        hipStream_t s) {
    const int64_t n = p->m.n;
    const int64_t col_bytes = static_cast<int64_t>(sizeof(double2)) * n * R;
    const int m = gmres_restart(n, R, o);
    double2 *V1 = static_cast<double2 *>(p->V.get(static_cast<size_t>(col_bytes) * (m + 1)));
    Recycle first;            // space of the first cycle, deflates every later cycle
    BlockRecycle bfirst;      // the same for block GMRES
    DeflateCaps dcaps;        // block GMRES: its device buffers (sized at the first block cycle)
    double2 *bqk = nullptr, *bbm = nullptr;
    bool have_first = false;
    relres.assign(R, 0.0);
    std::vector<int32_t> all(R);
    for (int r = 0; r < R; ++r) all[r] = r;
    int32_t *act = static_cast<int32_t *>(p->act2.get(sizeof(int32_t) * R));
    double2 *blk = static_cast<double2 *>(p->r.get(sizeof(double2) * static_cast<size_t>(n) * R));
    double2 *Xa = static_cast<double2 *>(p->xa.get(sizeof(double2) * static_cast<size_t>(n) * R));
    double2 *AX = static_cast<double2 *>(p->axa.get(sizeof(double2) * static_cast<size_t>(n) * R));
    double2 *Rres = static_cast<double2 *>(p->rres.get(sizeof(double2) * static_cast<size_t>(n) * R));
    to_device(act, all, s);
    bblas_gather(n, R, act, b, ldb, blk, s);
    const std::vector<double> bn = column_norms(p, blk, R, s);
    bblas_gather(n, R, act, x, ldx, blk, s);
    const std::vector<double> xn = column_norms(p, blk, R, s);
    std::vector<char> xzero(R);
    std::vector<int32_t> active;
    for (int r = 0; r < R; ++r) {
        if (!std::isfinite(bn[r])) fail(VSIE_E_NAN, "right-hand side is not finite");
        if (!std::isfinite(xn[r])) fail(VSIE_E_NAN, "initial guess is not finite");
        xzero[r] = xn[r] == 0.0;
        if (bn[r] == 0.0) blas_zero(n, x + static_cast<int64_t>(r) * ldx, s);
        else active.push_back(r);
    }
    vsie_status status = VSIE_OK;
    while (!active.empty()) {
        const int na = static_cast<int>(active.size());
        to_device(act, active, s);
        bool any_x = false;
        for (int r : active) any_x = any_x || !xzero[r];
        if (any_x) {
            bblas_gather(n, na, act, x, ldx, Xa, s);
            apply_op_graph(p, f, VSIE_FP64, adjoint, na, Xa, n, AX, n, s);
            for (int r : active) cnt.mv64[r]++;
            bblas_sub(n, na, act, b, ldb, AX, Rres, s);
        } else {
            bblas_gather(n, na, act, b, ldb, Rres, s);
        }
        const std::vector<double> rn = column_norms(p, Rres, na, s);
        if (p->progress) {
            double worst = 0.0;
            for (int sl = 0; sl < na; ++sl) worst = std::max(worst, rn[sl] / bn[active[sl]]);
            std::fprintf(stderr, "[vsie] outer step %d: %d active columns, max FP64 relative residual %.3e\n",
                         cnt.outer[active[0]], na, worst);
            std::fflush(stderr);
        }
        std::vector<int32_t> next, keep_slot;
        std::vector<double> next_rn, next_tol;
        for (int sl = 0; sl < na; ++sl) {
            const int r = active[sl];
            if (!std::isfinite(rn[sl])) fail(VSIE_E_NAN, "non-finite residual");
            relres[r] = rn[sl] / bn[r];
            if (relres[r] <= o.tol) continue;
            if (cnt.it[r] >= o.max_iter || (prec == VSIE_FP32 && cnt.outer[r] >= o.max_outer)) {
                status = VSIE_E_NOCONV;
                continue;
            }
            double t = o.tol * bn[r] / rn[sl];
            if (prec == VSIE_FP32 && !(o.relax > 0 && !o.block)) t = std::max(t, o.inner_tol);
            next.push_back(r);
            keep_slot.push_back(sl);
            next_rn.push_back(rn[sl]);
            next_tol.push_back(t);
        }
        if (next.empty()) break;
        double2 *cyc_res = Rres;
        if (static_cast<int>(next.size()) != na) {  // compact the residual block
            to_device(act, keep_slot, s);
            bblas_gather(n, static_cast<int>(next.size()), act, Rres, n, Xa, s);
            cyc_res = Xa;
        }
        for (int r : next) cnt.outer[r]++;
        int done;
        if (o.block) {
            const int Ra = static_cast<int>(next.size());
            const int mb = block_restart(n, Ra, o);
            const size_t vbytes = sizeof(double2) * static_cast<size_t>(n) * Ra * (mb + 1);
            if (!dcaps.kcap) {
                dcaps = deflate_caps(R, [&](int w) { return block_restart(n, w, o); });
                bqk = static_cast<double2 *>(p->bqk.get(dcaps.qk));
                bbm = static_cast<double2 *>(p->bbm.get(dcaps.bm));
            }
            if (!have_first) {
                done = block_cycle(p, f, prec, adjoint, next, cyc_res, next_rn, next_tol, mb, o.max_iter, x, ldx,
                                   cnt, s, static_cast<double2 *>(p->V.get(vbytes)), &bfirst, nullptr, nullptr, bqk);
                have_first = true;
            } else {
                done = block_cycle(p, f, prec, adjoint, next, cyc_res, next_rn, next_tol, mb, o.max_iter, x, ldx,
                                   cnt, s, static_cast<double2 *>(p->V2.get(vbytes)), nullptr,
                                   bfirst.k > 0 ? &bfirst : nullptr, bbm, nullptr);
            }
        } else if (!have_first) {
            done = gmres_cycle(p, f, prec, adjoint, R, next, cyc_res, next_rn, next_tol, m, o.max_iter,
                               x, ldx, cnt, s, V1, &first, nullptr, o.relax);
            have_first = true;
        } else {
            double2 *V2 = static_cast<double2 *>(p->V2.get(static_cast<size_t>(col_bytes) * (m + 1)));
            done = gmres_cycle(p, f, prec, adjoint, R, next, cyc_res, next_rn, next_tol, m, o.max_iter,
                               x, ldx, cnt, s, V2, nullptr, &first, o.relax);
        }
        for (int r : next) xzero[r] = 0;
        if (done == 0) {  // breakdown at the first step for every rhs: no progress possible
            status = VSIE_E_NOCONV;
            break;
        }
        active = next;
    }
    return status;
}

// ---------------------------------------------------------------------------
// Block GMRES: one block Krylov space for all right-hand sides of a cycle.
//
// Block Arnoldi with classical Gram-Schmidt twice as complex GEMMs (rocBLAS
// zgemm, FP64 matrix cores), CholeskyQR2 for each new block, and an
// incremental Householder QR of the block upper Hessenberg matrix on the host
// (one reflector per column, Ra + 1 rows long) that yields each column's
// residual norm after every block step.

// G = T^H T with T upper triangular (G Hermitian r x r, column-major).  A
// diagonal shift is added when a pivot is not safely positive (a nearly
// rank-deficient block); the second CholeskyQR pass restores orthogonality.
void chol_upper(int r, const std::vector<cd> &G, std::vector<cd> &T) {
    double dmax = 0.0;
    for (int i = 0; i < r; ++i) dmax = std::max(dmax, G[static_cast<size_t>(i) * r + i].real());
    if (!(dmax > 0.0) || !std::isfinite(dmax)) fail(VSIE_E_NAN, "block QR: zero or non-finite block");
    for (double shift = 0.0;; shift = shift == 0.0 ? 1e-14 * dmax : shift * 100.0) {
        if (shift > 1e-4 * dmax) fail(VSIE_E_NAN, "block QR: Cholesky failed");
        T.assign(static_cast<size_t>(r) * r, 0.0);
        bool ok = true;
        for (int j = 0; j < r && ok; ++j) {
            for (int i = 0; i <= j; ++i) {
                cd acc = G[static_cast<size_t>(j) * r + i];
                if (i == j) acc += shift;
                for (int k = 0; k < i; ++k)
                    acc -= std::conj(T[static_cast<size_t>(i) * r + k]) * T[static_cast<size_t>(j) * r + k];
                if (i == j) {
                    if (!(acc.real() > 1e-15 * dmax)) {
                        ok = false;
                        break;
                    }
                    T[static_cast<size_t>(j) * r + j] = std::sqrt(acc.real());
                } else {
                    T[static_cast<size_t>(j) * r + i] = acc / T[static_cast<size_t>(i) * r + i];
                }
            }
        }
        if (ok) return;
    }
}

// inverse of an upper triangular r x r matrix (column-major)
void tri_inv_upper(int r, const std::vector<cd> &T, std::vector<cd> &Ti) {
    Ti.assign(static_cast<size_t>(r) * r, 0.0);
    for (int j = 0; j < r; ++j) {
        Ti[static_cast<size_t>(j) * r + j] = 1.0 / T[static_cast<size_t>(j) * r + j];
        for (int i = j - 1; i >= 0; --i) {
            cd acc = 0.0;
            for (int k = i + 1; k <= j; ++k) acc += T[static_cast<size_t>(k) * r + i] * Ti[static_cast<size_t>(j) * r + k];
            Ti[static_cast<size_t>(j) * r + i] = -acc / T[static_cast<size_t>(i) * r + i];
        }
    }
}

using zc = rocblas_double_complex;
inline const zc *zcp(const double2 *p) { return reinterpret_cast<const zc *>(p); }
inline zc *zcp(double2 *p) { return reinterpret_cast<zc *>(p); }

// C = op(A) B with plain column-major operands (rocBLAS zgemm)
void zgemm(vsie_problem *p, bool conjA, int64_t m, int64_t nn, int64_t k, cd alpha, const double2 *A,
           int64_t lda, const double2 *B, int64_t ldb, cd beta, double2 *C, int64_t ldc) {
    require(m <= INT32_MAX && nn <= INT32_MAX && k <= INT32_MAX && lda <= INT32_MAX &&
                ldb <= INT32_MAX && ldc <= INT32_MAX,
            "block GEMM too large");
    const zc a{alpha.real(), alpha.imag()}, b{beta.real(), beta.imag()};
    check_blas(rocblas_zgemm(p->blas, conjA ? rocblas_operation_conjugate_transpose : rocblas_operation_none,
                             rocblas_operation_none, static_cast<rocblas_int>(m), static_cast<rocblas_int>(nn),
                             static_cast<rocblas_int>(k), &a, zcp(A), static_cast<rocblas_int>(lda), zcp(B),
                             static_cast<rocblas_int>(ldb), &b, zcp(C), static_cast<rocblas_int>(ldc)),
               "rocblas_zgemm");
}

// C = A^H B for tall A (k x m) and B (k x nn), k >> m, nn.  A single GEMM
// would give only ceil(m/64) ceil(nn/64) output tiles, each running the whole
// k loop, so the rows are cut into slabs: one strided-batched GEMM makes the
// product of every slab, a second call the ragged last slab, and the slab
// partials are summed in slab order (deterministic).
constexpr int64_t kTallTargetTiles = 2048;
constexpr int64_t kTallMinSlab = 512;

int64_t tall_slabs(int64_t m, int64_t nn, int64_t k) {
    const int64_t tiles = ((m + 63) / 64) * ((nn + 63) / 64);
    return std::min((kTallTargetTiles + tiles - 1) / tiles, std::max<int64_t>(1, k / kTallMinSlab));
}
// bytes of the slab partials of zgemm_tall_cn (0 when one GEMM does it)
size_t tall_bytes(int64_t m, int64_t nn, int64_t k) {
    if (nn <= kTsMaxCols) return ts_cn_bytes(m, nn, k);
    const int64_t slabs = tall_slabs(m, nn, k);
    if (slabs <= 1) return 0;
    const int64_t rows = (k + slabs - 1) / slabs;
    const int64_t full = k / rows, tail = k - full * rows;
    return sizeof(double2) * static_cast<size_t>(m * nn * (full + (tail > 0 ? 1 : 0)));
}

void zgemm_tall_cn(vsie_problem *p, int64_t m, int64_t nn, int64_t k, const double2 *A, int64_t lda,
                   const double2 *B, int64_t ldb, double2 *C, int64_t ldc, hipStream_t s) {
    if (nn <= kTsMaxCols) {
        // blocks of few columns: the hand-written slab kernel (rocBLAS tiles are
        // 64 columns wide and would leave most of each tile empty)
        double2 *P = static_cast<double2 *>(p->bsk.get(ts_cn_bytes(m, nn, k)));
        ts_cn(k, m, nn, A, lda, B, ldb, P, C, ldc, s);
        return;
    }
    const int64_t slabs = tall_slabs(m, nn, k);
    if (slabs <= 1) {
        zgemm(p, true, m, nn, k, 1.0, A, lda, B, ldb, 0.0, C, ldc);
        return;
    }
    const int64_t rows = (k + slabs - 1) / slabs;
    const int64_t full = k / rows, tail = k - full * rows;
    const int parts = static_cast<int>(full + (tail > 0 ? 1 : 0));
    const int64_t cnt = m * nn;
    double2 *P = static_cast<double2 *>(p->bsk.get(sizeof(double2) * static_cast<size_t>(cnt) * parts));
    require(m <= INT32_MAX && nn <= INT32_MAX && rows <= INT32_MAX && lda <= INT32_MAX && ldb <= INT32_MAX,
            "block GEMM too large");
    const zc one{1.0, 0.0}, zero{0.0, 0.0};
    check_blas(rocblas_zgemm_strided_batched(
                   p->blas, rocblas_operation_conjugate_transpose, rocblas_operation_none,
                   static_cast<rocblas_int>(m), static_cast<rocblas_int>(nn), static_cast<rocblas_int>(rows), &one,
                   zcp(A), static_cast<rocblas_int>(lda), rows, zcp(B), static_cast<rocblas_int>(ldb), rows, &zero,
                   zcp(P), static_cast<rocblas_int>(m), cnt, static_cast<rocblas_int>(full)),
               "rocblas_zgemm_strided_batched");
    if (tail > 0)
        zgemm(p, true, m, nn, tail, 1.0, A + full * rows, lda, B + full * rows, ldb, 0.0, P + full * cnt, m);
    blas_sum_slabs(m, nn, parts, P, C, ldc, s);
}

// C = alpha A B + beta C for tall A (n x k) and a block of nn columns: the
// hand-written kernel for nn <= kTsMaxCols (alpha = 1 or -1, beta = 0 or 1,
// the only forms the block solver uses), rocBLAS otherwise.
void zgemm_tall_nn(vsie_problem *p, int64_t n, int64_t nn, int64_t k, double alpha, const double2 *A, int64_t lda,
                   const double2 *B, int64_t ldb, double beta, double2 *C, int64_t ldc, hipStream_t s) {
    if (nn <= kTsMaxCols && (alpha == 1.0 || alpha == -1.0) && (beta == 0.0 || beta == 1.0)) {
        ts_nn(n, k, nn, alpha, beta == 1.0, A, lda, B, ldb, C, ldc, s);
        return;
    }
    zgemm(p, false, n, nn, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

// CholeskyQR2 of the n x r block Wsrc: dst = Wsrc T^{-1} with orthonormal
// columns and T upper triangular (host).  tmp is an n x r scratch block.
void cholqr2(vsie_problem *p, int64_t n, int r, const double2 *Wsrc, double2 *tmp, double2 *dst,
             std::vector<cd> &T, hipStream_t s) {
    double2 *Gd = static_cast<double2 *>(p->bg.get(sizeof(double2) * static_cast<size_t>(r) * r));
    std::vector<double2> gh;
    std::vector<cd> G(static_cast<size_t>(r) * r), T1, T2, Ti;
    const double2 *src = Wsrc;
    for (int pass = 0; pass < 2; ++pass) {
        double2 *out = pass == 0 ? tmp : dst;
        zgemm_tall_cn(p, r, r, n, src, n, src, n, Gd, r, s);
        to_host(gh, Gd, static_cast<size_t>(r) * r, s);
        for (size_t t = 0; t < G.size(); ++t) G[t] = cd(gh[t].x, gh[t].y);
        std::vector<cd> &Tp = pass == 0 ? T1 : T2;
        chol_upper(r, G, Tp);
        tri_inv_upper(r, Tp, Ti);
        std::vector<double2> th(Ti.size());
        for (size_t t = 0; t < Ti.size(); ++t) th[t] = make_double2(Ti[t].real(), Ti[t].imag());
        to_device(Gd, th, s);
        zgemm_tall_nn(p, n, r, r, 1.0, src, n, Gd, r, 0.0, out, n, s);
        src = out;
    }
    // T = T2 T1
    T.assign(static_cast<size_t>(r) * r, 0.0);
    for (int j = 0; j < r; ++j)
        for (int i = 0; i <= j; ++i) {
            cd acc = 0.0;
            for (int k = i; k <= j; ++k) acc += T2[static_cast<size_t>(k) * r + i] * T1[static_cast<size_t>(j) * r + k];
            T[static_cast<size_t>(j) * r + i] = acc;
        }
}

// CholeskyQR2 of the n x r block Wsrc entirely on the device (r <= kSmallChol):
// dst = Wsrc T^{-1}; T = T2 T1 goes to Tdev (r x r) and the two passes'
// status words to status[0], status[1] (0: factorised; see small_chol_kernel).
// Nothing is copied to the host: the caller reads T and the status together
// with the step's other coefficients.
void cholqr2_dev(vsie_problem *p, int64_t n, int r, const double2 *Wsrc, double2 *tmp, double2 *dst, double2 *Tdev,
                 int *status, hipStream_t s) {
    const int64_t rr = static_cast<int64_t>(r) * r;
    double2 *buf = static_cast<double2 *>(p->bg.get(sizeof(double2) * static_cast<size_t>(5 * rr)));
    double2 *G = buf, *T1 = buf + rr, *Ti = buf + 2 * rr, *T2 = buf + 3 * rr;
    zgemm_tall_cn(p, r, r, n, Wsrc, n, Wsrc, n, G, r, s);
    launch_small_chol(G, r, T1, Ti, nullptr, nullptr, status, s);
    zgemm_tall_nn(p, n, r, r, 1.0, Wsrc, n, Ti, r, 0.0, tmp, n, s);
    zgemm_tall_cn(p, r, r, n, tmp, n, tmp, n, G, r, s);
    launch_small_chol(G, r, T2, Ti, T1, Tdev, status + 1, s);
    zgemm_tall_nn(p, n, r, r, 1.0, tmp, n, Ti, r, 0.0, dst, n, s);
}

// The host's reading of the two status words of cholqr2_dev.
void check_chol_status(const int *st) {
    for (int q = 0; q < 2; ++q) {
        if (st[q] == 1) fail(VSIE_E_NAN, "block QR: zero or non-finite block");
        if (st[q] != 0) fail(VSIE_E_NAN, "block QR: Cholesky failed");
    }
}

// Householder reflector P = I - 2 u u^H / (u^H u) with P x = alpha e_1; u overwrites x.
// Returns u^H u (0 when x = 0: P = I).
double make_reflector(cd *x, int len, cd &alpha) {
    double nx = 0.0;
    for (int i = 0; i < len; ++i) nx += std::norm(x[i]);
    nx = std::sqrt(nx);
    if (nx == 0.0) {
        alpha = 0.0;
        return 0.0;
    }
    const cd ph = std::abs(x[0]) > 0.0 ? x[0] / std::abs(x[0]) : cd(1.0, 0.0);
    alpha = -ph * nx;
    x[0] -= alpha;
    double uu = 0.0;
    for (int i = 0; i < len; ++i) uu += std::norm(x[i]);
    return uu;
}

// y <- (I - 2 u u^H / uu) y for vectors of length len.  Written on the real
// and imaginary parts (std::complex stores them interleaved) so that the
// compiler vectorises both loops: the block QR applies thousands of these
// per column and step.
inline void apply_reflector(const cd *u, double uu, int len, cd *y) {
    if (uu == 0.0) return;
    const double *ur = reinterpret_cast<const double *>(u);
    double *yr = reinterpret_cast<double *>(y);
    double sr = 0.0, si = 0.0;  // u^H y
    for (int i = 0; i < len; ++i) {
        const double a = ur[2 * i], b = ur[2 * i + 1], c = yr[2 * i], e = yr[2 * i + 1];
        sr += a * c + b * e;
        si += a * e - b * c;
    }
    const double f = 2.0 / uu;
    sr *= f;
    si *= f;
    for (int i = 0; i < len; ++i) {
        const double a = ur[2 * i], b = ur[2 * i + 1];
        yr[2 * i] -= sr * a - si * b;
        yr[2 * i + 1] -= sr * b + si * a;
    }
}

// One block GMRES cycle for the right-hand sides rhs[0..Ra) with residual
// block Rres (n x Ra, column norms rn) and per-column tolerances, driven one
// block step at a time so that the cycles of several frequencies can share
// one operator launch per step: begin(); then, while wants_product(), the
// caller writes op(A) input() to output() and calls after_product(); finally
// finish() adds the corrections to x and returns the number of block steps.
// V holds the basis (n x Ra (m + 1)); W (n x Ra) receives each product and is
// overwritten by the step.  The shared work buffers (Z, the block Hessenberg
// column, the Gram matrix, the slab partials, the deflation coefficients and
// the column index array) are taken from the problem at each use, so cycles
// of several frequencies advanced one after another on one stream can share
// them.
// Entries (double2) of the per-step stage of small-block cycles: two
// Gram-Schmidt coefficient blocks, the R block and the status words.
inline size_t stage_len(int64_t ldH, int Ra) {
    return static_cast<size_t>(2 * ldH * Ra + static_cast<int64_t>(Ra) * Ra + 1);
}

class BlockCycle {
  public:
    // Bm: device C^H A V of this cycle (kr x m Ra, used when use holds a
    // space); qk: device memory for the Q E of the space this cycle keeps in
    // save (kBlockRecycleMax x (kBlockRecycleMax + Ra) at most)
    BlockCycle(vsie_problem *p, int f, vsie_precision prec, std::vector<int32_t> rhs, double2 *Rres,
               std::vector<double> rn, std::vector<double> ctol, int m, int iter_cap, double2 *x, int64_t ldx,
               SolveCounters &cnt, hipStream_t s, double2 *V, double2 *W, BlockRecycle *save,
               const BlockRecycle *use, double2 *Bm, double2 *qk, bool report)
        : p_(p), f_(f), prec_(prec), rhs_(std::move(rhs)), Rres_(Rres), rn_(std::move(rn)),
          ctol_(std::move(ctol)), m_(m), iter_cap_(iter_cap), x_(x), ldx_(ldx), cnt_(cnt), s_(s), V_(V), W_(W),
          save_(save), use_(use), Bm_(Bm), qk_(qk), report_(report), n_(p->m.n), Ra_(static_cast<int>(rhs_.size())),
          ldH_(static_cast<int64_t>(m + 1) * Ra_), kr_(use ? use->k : 0), kv_(use ? use->k + use->Ra : 0) {}

    void begin();
    bool wants_product() const {
        if (done_ || j_ >= m_) return false;
        for (int r : rhs_)
            if (cnt_.it[r] >= iter_cap_) return false;
        return true;
    }
    const double2 *input() const { return V_ + static_cast<int64_t>(j_) * Ra_ * n_; }
    double2 *output() const { return W_; }
    int width() const { return Ra_; }
    int freq() const { return f_; }
    void after_product() {
        step_device();
        step_host();
    }
    // after_product in two halves: the device work of the step (Gram-Schmidt
    // and CholeskyQR; the next basis block is queued when it returns) and the
    // host's QR of the block Hessenberg with the convergence test.  Between
    // them the caller may queue the next step's product on input_ahead()
    // when lookahead_ok(): the host QR then overlaps the product.
    void step_device();
    void step_host();
    bool lookahead_ok() const;
    const double2 *input_ahead() const { return V_ + static_cast<int64_t>(j_ + 1) * Ra_ * n_; }
    int finish();
    void add_operator_seconds(double t) { sec_[0] += t; }
    // largest residual estimate after the last step, relative to the cycle start
    double worst() const { return worst_; }

  private:
    using clk = std::chrono::steady_clock;
    double2 *Dd() const { return static_cast<double2 *>(p_->brc.get(sizeof(double2) * static_cast<size_t>(kv_) * Ra_)); }
    double2 *Zt() const { return static_cast<double2 *>(p_->bzt.get(sizeof(double2) * static_cast<size_t>(kr_) * Ra_)); }
    // small blocks: both Gram-Schmidt passes' coefficients (ldH_ x Ra each),
    // the new R block (Ra x Ra) and two status words, brought to the host in
    // one copy per step
    bool dev_qr() const { return Ra_ <= kSmallChol; }
    double2 *stage() const {
        return static_cast<double2 *>(p_->bst.get(sizeof(double2) * stage_len(ldH_, Ra_)));
    }
    int32_t *act() const {
        int32_t *a = static_cast<int32_t *>(p_->act.get(sizeof(int32_t) * Ra_));
        to_device(a, rhs_, s_);
        return a;
    }
    // progress mode: wall time of the sections of each block step (the stream
    // is synchronised at each mark, so these runs are diagnostic)
    void mark(clk::time_point &t, int which) {
        if (!p_->progress) return;
        VSIE_HIP(hipStreamSynchronize(s_));
        const clk::time_point now = clk::now();
        sec_[which] += std::chrono::duration<double>(now - t).count();
        t = now;
    }

    vsie_problem *p_;
    int f_;
    vsie_precision prec_;
    std::vector<int32_t> rhs_;
    double2 *Rres_;
    std::vector<double> rn_, ctol_;
    int m_, iter_cap_;
    double2 *x_;
    int64_t ldx_;
    SolveCounters &cnt_;
    hipStream_t s_;
    double2 *V_, *W_;
    BlockRecycle *save_;
    const BlockRecycle *use_;
    double2 *Bm_, *qk_;
    bool report_;
    int64_t n_;
    int Ra_;
    int64_t ldH_, kr_, kv_;
    // transformed right-hand sides (column-major, ldH_ rows), the R factor of
    // the block Hessenberg packed by columns and grown one block column per
    // step (the full (m Ra)^2 array would be several GB to zero), and one
    // Householder reflector per column (Ra + 1 long, at c (Ra + 1))
    std::vector<cd> G_, Rf_, U_;
    std::vector<double> UU_;
    int j_ = 0, jdone_ = 0;
    bool done_ = false;
    double worst_ = 1.0;
    double sec_[4] = {0, 0, 0, 0};  // operator, Gram-Schmidt, CholeskyQR, host QR
    // the step's new block column of the Hessenberg matrix and R block, from
    // step_device to step_host
    std::vector<cd> Hc_, T_;
    clk::time_point tm_;
};

void BlockCycle::begin() {
    if (!p_->blas) check_blas(rocblas_create_handle(&p_->blas), "rocblas_create_handle");
    check_blas(rocblas_set_stream(p_->blas, s_), "rocblas_set_stream");
    // deflation by an earlier cycle's space (C = V Qk, U = V_k R^{-1}):
    // z = C^H r, r -= C z, x += U z; later Bm = C^H A v for every new basis
    // column (column-major, kr rows, on the device)
    if (kr_ > 0) {
        double2 *D = Dd(), *Z = Zt();
        zgemm_tall_cn(p_, kv_, Ra_, n_, use_->V, n_, Rres_, n_, D, kv_, s_);
        zgemm(p_, true, kr_, Ra_, kv_, 1.0, use_->Qk, kv_, D, kv_, 0.0, Z, kr_);
        zgemm(p_, false, kv_, Ra_, kr_, 1.0, use_->Qk, kv_, Z, kr_, 0.0, D, kv_);
        zgemm_tall_nn(p_, n_, Ra_, kv_, -1.0, use_->V, n_, D, kv_, 1.0, Rres_, n_, s_);
        std::vector<double2> zh;
        to_host(zh, Z, static_cast<size_t>(kr_) * Ra_, s_);
        std::vector<cd> z(zh.size());
        for (size_t q = 0; q < z.size(); ++q) z[q] = cd(zh[q].x, zh[q].y);
        tri_solve_upper_cols(use_->R.data(), kr_, kr_, Ra_, z.data());
        for (size_t q = 0; q < z.size(); ++q) zh[q] = make_double2(z[q].real(), z[q].imag());
        to_device(D, zh, s_);
        zgemm_tall_nn(p_, n_, Ra_, kr_, 1.0, use_->V, n_, D, kr_, 0.0, W_, n_, s_);
        blas_scatter_add(n_, Ra_, act(), W_, x_, ldx_, s_);
    }
    std::vector<cd> S0;
    double2 *Z = static_cast<double2 *>(p_->ax.get(sizeof(double2) * static_cast<size_t>(n_) * Ra_));
    if (dev_qr()) {
        const int64_t rr = static_cast<int64_t>(Ra_) * Ra_;
        double2 *st = stage();
        cholqr2_dev(p_, n_, Ra_, Rres_, Z, V_, st, reinterpret_cast<int *>(st + rr), s_);
        std::vector<double2> h;
        to_host(h, st, static_cast<size_t>(rr + 1), s_);
        check_chol_status(reinterpret_cast<const int *>(h.data() + rr));
        S0.resize(static_cast<size_t>(rr));
        for (int64_t q = 0; q < rr; ++q) S0[q] = cd(h[q].x, h[q].y);
    } else {
        cholqr2(p_, n_, Ra_, Rres_, Z, V_, S0, s_);
    }
    G_.assign(static_cast<size_t>(ldH_) * Ra_, 0.0);
    for (int c = 0; c < Ra_; ++c)
        for (int i = 0; i <= c; ++i) G_[static_cast<size_t>(c) * ldH_ + i] = S0[static_cast<size_t>(c) * Ra_ + i];
    U_.assign(static_cast<size_t>(m_) * Ra_ * (Ra_ + 1), 0.0);
    UU_.assign(static_cast<size_t>(m_) * Ra_, 0.0);
}

void BlockCycle::step_device() {
    const int j = j_;
    const int Ra = Ra_;
    const int64_t n = n_, kr = kr_, kv = kv_;
    clk::time_point &tm = tm_;
    tm = clk::now();
    for (int r : rhs_) (prec_ == VSIE_FP64 ? cnt_.mv64 : cnt_.mv32)[r]++;
    const int64_t kb = static_cast<int64_t>(j + 1) * Ra;
    double2 *W = W_;
    std::vector<cd> &Hc = Hc_;
    Hc.assign(static_cast<size_t>(kb + Ra) * Ra, 0.0);  // new block column, rows 0..kb+Ra
    std::vector<double2> hh;
    for (int pass = 0; pass < 2; ++pass) {
        if (kr > 0) {
            // D = V^H W, z = Qk^H D (summed over both passes into this step's
            // block of Bm), W -= V (Qk z)
            double2 *D = Dd();
            double2 *Bj = Bm_ + static_cast<int64_t>(j) * Ra * kr;
            zgemm_tall_cn(p_, kv, Ra, n, use_->V, n, W, n, D, kv, s_);
            zgemm(p_, true, kr, Ra, kv, 1.0, use_->Qk, kv, D, kv, pass == 0 ? 0.0 : 1.0, Bj, kr);
            const double2 *zp = Bj;
            if (pass == 1) {
                double2 *Z = Zt();
                zgemm(p_, true, kr, Ra, kv, 1.0, use_->Qk, kv, D, kv, 0.0, Z, kr);
                zp = Z;
            }
            zgemm(p_, false, kv, Ra, kr, 1.0, use_->Qk, kv, zp, kr, 0.0, D, kv);
            zgemm_tall_nn(p_, n, Ra, kv, -1.0, use_->V, n, D, kv, 1.0, W, n, s_);
        }
        if (dev_qr()) {  // this pass's coefficients stay in the stage until the step's one copy
            double2 *Hd = stage() + static_cast<int64_t>(pass) * kb * Ra;
            zgemm_tall_cn(p_, kb, Ra, n, V_, n, W, n, Hd, kb, s_);
            zgemm_tall_nn(p_, n, Ra, kb, -1.0, V_, n, Hd, kb, 1.0, W, n, s_);
            continue;
        }
        double2 *Hd = static_cast<double2 *>(p_->bh.get(sizeof(double2) * static_cast<size_t>(ldH_) * Ra));
        zgemm_tall_cn(p_, kb, Ra, n, V_, n, W, n, Hd, kb, s_);
        zgemm_tall_nn(p_, n, Ra, kb, -1.0, V_, n, Hd, kb, 1.0, W, n, s_);
        to_host(hh, Hd, static_cast<size_t>(kb) * Ra, s_);
        for (int c = 0; c < Ra; ++c)
            for (int64_t i = 0; i < kb; ++i)
                Hc[static_cast<size_t>(c) * (kb + Ra) + i] += cd(hh[c * kb + i].x, hh[c * kb + i].y);
    }
    mark(tm, 1);
    std::vector<cd> &T = T_;
    double2 *Z = static_cast<double2 *>(p_->ax.get(sizeof(double2) * static_cast<size_t>(n) * Ra));
    if (dev_qr()) {
        const int64_t hb = kb * Ra, rr = static_cast<int64_t>(Ra) * Ra;
        double2 *st = stage();
        cholqr2_dev(p_, n, Ra, W, Z, V_ + kb * n, st + 2 * hb, reinterpret_cast<int *>(st + 2 * hb + rr), s_);
        to_host(hh, st, static_cast<size_t>(2 * hb + rr + 1), s_);
        check_chol_status(reinterpret_cast<const int *>(hh.data() + 2 * hb + rr));
        for (int c = 0; c < Ra; ++c)
            for (int64_t i = 0; i < kb; ++i) {
                const double2 a = hh[c * kb + i], b = hh[hb + c * kb + i];
                Hc[static_cast<size_t>(c) * (kb + Ra) + i] = cd(a.x + b.x, a.y + b.y);
            }
        T.resize(static_cast<size_t>(rr));
        for (int64_t q = 0; q < rr; ++q) T[q] = cd(hh[2 * hb + q].x, hh[2 * hb + q].y);
    } else {
        cholqr2(p_, n, Ra, W, Z, V_ + kb * n, T, s_);
    }
    mark(tm, 2);
}

// A step whose residual estimate (the previous step's) is still this far above
// the tolerance is not expected to end the cycle, so the next product may be
// queued before the host QR; a wrong guess only costs the unused product.
constexpr double kLookaheadMargin = 1e3;

bool BlockCycle::lookahead_ok() const {
    if (p_->progress || j_ + 1 >= m_) return false;
    for (int r : rhs_)
        if (cnt_.it[r] + 1 >= iter_cap_) return false;
    double tmax = 0.0;
    for (double t : ctol_) tmax = std::max(tmax, t);
    return worst_ > kLookaheadMargin * tmax;
}

void BlockCycle::step_host() {
    const int j = j_;
    const int Ra = Ra_;
    const int64_t kb = static_cast<int64_t>(j + 1) * Ra;
    clk::time_point &tm = tm_;
    std::vector<cd> &Hc = Hc_;
    const std::vector<cd> &T = T_;
    for (int c = 0; c < Ra; ++c)
        for (int i = 0; i <= c; ++i) Hc[static_cast<size_t>(c) * (kb + Ra) + kb + i] = T[static_cast<size_t>(c) * Ra + i];
    // previous reflectors on the new columns (independent per column)
    const int64_t c0 = static_cast<int64_t>(j) * Ra;
    parallel_for(Ra, 8.0 * Ra * c0 * (Ra + 1), [&](int c) {
        cd *h = &Hc[static_cast<size_t>(c) * (kb + Ra)];
        for (int64_t k = 0; k < c0; ++k) apply_reflector(&U_[static_cast<size_t>(k) * (Ra + 1)], UU_[k], Ra + 1, h + k);
    });
    // this block's reflectors, column by column
    Rf_.resize(packed_col(c0 + Ra));
    for (int cl = 0; cl < Ra; ++cl) {
        const int64_t c = c0 + cl;
        cd *h = &Hc[static_cast<size_t>(cl) * (kb + Ra)];
        for (int64_t k = c0; k < c; ++k) apply_reflector(&U_[static_cast<size_t>(k) * (Ra + 1)], UU_[k], Ra + 1, h + k);
        cd *u = &U_[static_cast<size_t>(c) * (Ra + 1)];
        for (int t = 0; t <= Ra; ++t) u[t] = h[c + t];
        cd alpha;
        UU_[c] = make_reflector(u, Ra + 1, alpha);
        cd *rc_ = &Rf_[packed_col(c)];
        for (int64_t i = 0; i < c; ++i) rc_[i] = h[i];
        rc_[c] = UU_[c] == 0.0 ? h[c] : alpha;
    }
    // the same reflectors, in order, on the transformed right-hand sides
    // (independent per column; they do not feed back into the reflectors)
    parallel_for(Ra, 8.0 * Ra * Ra * (Ra + 1), [&](int rc) {
        for (int cl = 0; cl < Ra; ++cl) {
            const int64_t c = c0 + cl;
            apply_reflector(&U_[static_cast<size_t>(c) * (Ra + 1)], UU_[c], Ra + 1, &G_[static_cast<size_t>(rc) * ldH_ + c]);
        }
    });
    mark(tm, 3);
    for (int r : rhs_) cnt_.it[r]++;
    jdone_ = j + 1;
    j_ = j + 1;
    bool all = true;
    worst_ = 0.0;
    for (int rc = 0; rc < Ra; ++rc) {
        double res = 0.0;
        for (int t = 0; t < Ra; ++t) res += std::norm(G_[static_cast<size_t>(rc) * ldH_ + kb + t]);
        if (!std::isfinite(res)) fail(VSIE_E_NAN, "non-finite block residual");
        all = all && std::sqrt(res) <= ctol_[rc] * rn_[rc];
        worst_ = std::max(worst_, std::sqrt(res) / rn_[rc]);
    }
    if (p_->progress && report_) {
        std::fprintf(stderr,
                     "[vsie] block step %d (%d columns): max residual estimate %.3e of the cycle start "
                     "(seconds so far: operator %.3f, Gram-Schmidt %.3f, CholeskyQR %.3f, host QR %.3f)\n",
                     j + 1, Ra, worst_, sec_[0], sec_[1], sec_[2], sec_[3]);
        std::fflush(stderr);
    }
    done_ = all;
}

int BlockCycle::finish() {
    if (jdone_ == 0) return 0;
    const int Ra = Ra_;
    const int64_t n = n_, kr = kr_;
    // Y = R^{-1} G(0 : jdone Ra, :); with deflation also Wc = R_use^{-1} (Bm Y),
    // the coefficients of U (Bm Y) in the recycled basis
    const int64_t kk = static_cast<int64_t>(jdone_) * Ra;
    std::vector<cd> Ycol(static_cast<size_t>(kk) * Ra);
    for (int rc = 0; rc < Ra; ++rc)
        std::copy(G_.begin() + static_cast<size_t>(rc) * ldH_, G_.begin() + static_cast<size_t>(rc) * ldH_ + kk,
                  Ycol.begin() + static_cast<size_t>(rc) * kk);
    tri_solve_upper_cols_by([&](int64_t i) { return Rf_.data() + packed_col(i); }, kk, Ra, Ycol.data());
    std::vector<double2> Yh(static_cast<size_t>(kk) * Ra);
    for (size_t q = 0; q < Yh.size(); ++q) Yh[q] = make_double2(Ycol[q].real(), Ycol[q].imag());
    double2 *Yd = static_cast<double2 *>(p_->bh.get(sizeof(double2) * static_cast<size_t>(std::max(kk, ldH_)) * Ra));
    to_device(Yd, Yh, s_);
    std::vector<double2> Wc;
    if (kr > 0) {
        double2 *Z = Zt();
        zgemm(p_, false, kr, Ra, kk, 1.0, Bm_, kr, Yd, kk, 0.0, Z, kr);
        to_host(Wc, Z, static_cast<size_t>(kr) * Ra, s_);
        std::vector<cd> by(Wc.size());
        for (size_t q = 0; q < by.size(); ++q) by[q] = cd(Wc[q].x, Wc[q].y);
        tri_solve_upper_cols(use_->R.data(), kr, kr, Ra, by.data());
        for (size_t q = 0; q < Wc.size(); ++q) Wc[q] = make_double2(by[q].real(), by[q].imag());
    }
    zgemm_tall_nn(p_, n, Ra, kk, 1.0, V_, n, Yd, kk, 0.0, W_, n, s_);
    if (kr > 0) {  // x += V y - U (Bm y)
        double2 *D = Dd();
        to_device(D, Wc, s_);
        zgemm_tall_nn(p_, n, Ra, kr, -1.0, use_->V, n, D, kr, 1.0, W_, n, s_);
    }
    blas_scatter_add(n, Ra, act(), W_, x_, ldx_, s_);
    VSIE_HIP(hipStreamSynchronize(s_));
    if (save_ && kk <= kBlockRecycleMax) {
        save_->V = V_;
        save_->Ra = Ra;
        save_->k = kk;
        save_->R.assign(static_cast<size_t>(kk) * kk, 0.0);
        for (int64_t c = 0; c < kk; ++c)
            for (int64_t i = 0; i <= c; ++i) save_->R[static_cast<size_t>(c) * kk + i] = Rf_[packed_col(c) + i];
        // Q E: column j is the reflectors j, j - 1, ..., 0 applied to e_j (the
        // later ones act on rows below j, where e_j is zero)
        const int64_t kv = kk + Ra;
        std::vector<double2> qh(static_cast<size_t>(kv) * kk);
        parallel_for(static_cast<int>(kk), 4.0 * kk * kk * (Ra + 1), [&](int j) {
            std::vector<cd> v(kv, 0.0);
            v[j] = 1.0;
            for (int64_t c = j; c >= 0; --c)
                apply_reflector(&U_[static_cast<size_t>(c) * (Ra + 1)], UU_[c], Ra + 1, &v[c]);
            for (int64_t i = 0; i < kv; ++i)
                qh[static_cast<size_t>(j) * kv + i] = make_double2(v[i].real(), v[i].imag());
        });
        to_device(qk_, qh, s_);
        save_->Qk = qk_;
    } else if (save_) {
        save_->k = 0;
    }
    return jdone_;
}

// One block GMRES cycle of one frequency (the product of each step is one
// operator application of width Ra into the problem's W buffer).
int block_cycle(vsie_problem *p, int f, vsie_precision prec, bool adjoint, const std::vector<int32_t> &rhs,
                double2 *Rres, const std::vector<double> &rn, const std::vector<double> &ctol, int m,
                int iter_cap, double2 *x, int64_t ldx, SolveCounters &cnt, hipStream_t s, double2 *V,
                BlockRecycle *save, const BlockRecycle *use, double2 *Bm, double2 *qk) {
    const int64_t n = p->m.n;
    const int Ra = static_cast<int>(rhs.size());
    double2 *W = static_cast<double2 *>(p->w.get(sizeof(double2) * static_cast<size_t>(n) * Ra));
    BlockCycle c(p, f, prec, rhs, Rres, rn, ctol, m, iter_cap, x, ldx, cnt, s, V, W, save, use, Bm, qk, true);
    c.begin();
    bool queued = false;  // the product of the current step is already on the stream
    while (c.wants_product()) {
        if (!queued) {
            const auto t0 = std::chrono::steady_clock::now();
            if (p->progress) VSIE_HIP(hipStreamSynchronize(s));
            apply_op(p, f, prec, adjoint, Ra, c.input(), n, c.output(), n, s);
            if (p->progress) {
                VSIE_HIP(hipStreamSynchronize(s));
                c.add_operator_seconds(std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
            }
        }
        c.step_device();
        // far from convergence, queue the next product before the host QR
        queued = c.lookahead_ok();
        if (queued) apply_op(p, f, prec, adjoint, Ra, c.input_ahead(), n, c.output(), n, s);
        c.step_host();
    }
    // a queued product the cycle did not use only wrote W
    return c.finish();
}

// ---------------------------------------------------------------------------
// Several frequencies solved in lockstep.  Each frequency runs its own block
// GMRES (with FP64 refinement for VSIE_FP32) exactly as a one-frequency block
// solve would; the processes share only the operator launches: every block
// step and every refinement residual applies the operators of all
// frequencies still iterating together.

// One forward operator application y = A_f x of width R (x, y: n x R,
// leading dimension n).
struct ProdItem {
    int f;
    int R;
    const double2 *x;
    double2 *y;
};

// The products of items (ascending f).  Each maximal run of consecutive
// frequencies with one width whose inputs and outputs lie at constant
// strides (outputs disjoint) is one multi-frequency launch per source class
// when a matrix-core path takes that width; anything else is one application
// per item.  Returns the number of applications issued.
int apply_items(vsie_problem *p, vsie_precision prec, const std::vector<ProdItem> &items, hipStream_t s) {
    const int64_t n = p->m.n;
    auto batchable = [&](const ProdItem &it) {
        if (prec == VSIE_FP32) return use_mfma(p, prec, it.R) && !p->dense[it.f].A;
        return use_mfma64(p, prec, it.R);
    };
    int launches = 0;
    size_t i = 0;
    while (i < items.size()) {
        const ProdItem &a = items[i];
        size_t j = i + 1;
        if (batchable(a)) {
            const int64_t xs = j < items.size() ? items[j].x - a.x : 0;
            const int64_t ys = j < items.size() ? items[j].y - a.y : 0;
            const int64_t blk = n * a.R;
            while (j < items.size()) {
                const ProdItem &b = items[j];
                const int64_t d = static_cast<int64_t>(j - i);
                if (b.f != a.f + d || b.R != a.R || !batchable(b) || xs <= 0 || ys < blk || b.x - a.x != d * xs ||
                    b.y - a.y != d * ys)
                    break;
                ++j;
            }
            const int nf = static_cast<int>(j - i);
            if (prec == VSIE_FP32) apply_forward_mfma(p, a.f, nf, a.R, a.x, n, xs, a.y, n, ys, s);
            else apply_forward_mfma64(p, a.f, nf, a.R, a.x, n, xs, a.y, n, ys, s);
        } else {
            apply_op(p, a.f, prec, false, a.R, a.x, n, a.y, n, s);
        }
        ++launches;
        i = j;
    }
    return launches;
}

// Block steps per cycle when nf frequencies iterate together: their nf bases
// share the Krylov budget of one solve (and the host R factor stays as in
// block_restart).
int multi_restart(int64_t n, int Ra, const vsie_solve_opts &o, int nf) { return block_restart(n * nf, Ra, o); }

// Columns of one frequency's basis region: enough for any block width up to R.
int64_t multi_basis_cols(int64_t n, int R, const vsie_solve_opts &o, int nf) {
    int64_t vcols = 0;
    for (int Ra = 1; Ra <= R; ++Ra)
        vcols = std::max<int64_t>(vcols, static_cast<int64_t>(Ra) * (multi_restart(n, Ra, o, nf) + 1));
    return vcols;
}

// Solve A_{f0+t} x_t = b_t for t < nf, R columns each (column t R + r of b
// and x).  Per frequency: counters, relative residuals and status.
void solve_multi_batch(vsie_problem *p, int f0, int nf, vsie_precision prec, int R, const double2 *b, int64_t ldb,
                       double2 *x, int64_t ldx, const vsie_solve_opts &o, std::vector<SolveCounters> &cnt,
                       std::vector<std::vector<double>> &relres, std::vector<vsie_status> &status, hipStream_t s) {
    const int64_t n = p->m.n;
    const size_t z = sizeof(double2);
    const int64_t blk = n * R;  // one frequency's n x R block
    const int64_t region = multi_basis_cols(n, R, o, nf) * n;
    double2 *Vb = static_cast<double2 *>(p->V.get(z * static_cast<size_t>(region) * nf));
    double2 *V2b = static_cast<double2 *>(p->V2.get(z * static_cast<size_t>(region) * nf));
    double2 *Wb = static_cast<double2 *>(p->w.get(z * static_cast<size_t>(blk) * nf));
    double2 *Xa = static_cast<double2 *>(p->xa.get(z * static_cast<size_t>(blk) * nf));
    double2 *AX = static_cast<double2 *>(p->axa.get(z * static_cast<size_t>(blk) * nf));
    double2 *Rres = static_cast<double2 *>(p->rres.get(z * static_cast<size_t>(blk) * nf));
    double2 *tmp = static_cast<double2 *>(p->r.get(z * static_cast<size_t>(blk)));
    const DeflateCaps dc = deflate_caps(R, [&](int Ra) { return multi_restart(n, Ra, o, nf); });
    double2 *Qb = static_cast<double2 *>(p->bqk.get(dc.qk * nf));
    double2 *Bb = static_cast<double2 *>(p->bbm.get(dc.bm * nf));
    const int64_t qk_stride = static_cast<int64_t>(dc.qk / sizeof(double2));
    const int64_t bm_stride = static_cast<int64_t>(dc.bm / sizeof(double2));
    int32_t *act = static_cast<int32_t *>(p->act2.get(sizeof(int32_t) * R));
    auto bcol = [&](int t) { return b + static_cast<int64_t>(t) * R * ldb; };
    auto xcol = [&](int t) { return x + static_cast<int64_t>(t) * R * ldx; };

    struct Freq {
        std::vector<double> bn;
        std::vector<char> xzero;
        std::vector<int32_t> active;
        BlockRecycle first;  // first cycle's space, deflates the later cycles
        bool have_first = false;
    };
    std::vector<Freq> F(nf);
    std::vector<int32_t> all(R);
    for (int r = 0; r < R; ++r) all[r] = r;
    to_device(act, all, s);
    for (int t = 0; t < nf; ++t) {
        Freq &q = F[t];
        relres[t].assign(R, 0.0);
        status[t] = VSIE_OK;
        bblas_gather(n, R, act, bcol(t), ldb, tmp, s);
        q.bn = column_norms(p, tmp, R, s);
        bblas_gather(n, R, act, xcol(t), ldx, tmp, s);
        const std::vector<double> xn = column_norms(p, tmp, R, s);
        q.xzero.assign(R, 0);
        for (int r = 0; r < R; ++r) {
            if (!std::isfinite(q.bn[r])) fail(VSIE_E_NAN, "right-hand side is not finite");
            if (!std::isfinite(xn[r])) fail(VSIE_E_NAN, "initial guess is not finite");
            q.xzero[r] = xn[r] == 0.0;
            if (q.bn[r] == 0.0) blas_zero(n, xcol(t) + static_cast<int64_t>(r) * ldx, s);
            else q.active.push_back(r);
        }
    }
    for (;;) {
        // FP64 residuals r = b - A x of every frequency's active columns
        // (frequency t's block at offset t n R of Xa, AX and Rres)
        std::vector<ProdItem> items;
        std::vector<int> live;
        for (int t = 0; t < nf; ++t) {
            Freq &q = F[t];
            if (q.active.empty()) continue;
            live.push_back(t);
            const int na = static_cast<int>(q.active.size());
            bool any_x = false;
            for (int r : q.active) any_x = any_x || !q.xzero[r];
            to_device(act, q.active, s);
            if (any_x) {
                bblas_gather(n, na, act, xcol(t), ldx, Xa + t * blk, s);
                items.push_back({f0 + t, na, Xa + t * blk, AX + t * blk});
            } else {
                bblas_gather(n, na, act, bcol(t), ldb, Rres + t * blk, s);
            }
        }
        if (live.empty()) break;
        apply_items(p, VSIE_FP64, items, s);
        for (const ProdItem &it : items) {
            const int t = it.f - f0;
            for (int r : F[t].active) cnt[t].mv64[r]++;
            to_device(act, F[t].active, s);
            bblas_sub(n, it.R, act, bcol(t), ldb, AX + t * blk, Rres + t * blk, s);
        }
        // the cycles of this refinement step
        std::vector<std::unique_ptr<BlockCycle>> cyc(nf);
        std::vector<std::vector<int32_t>> next(nf);
        double worst_start = 0.0;
        for (int t : live) {
            Freq &q = F[t];
            const int na = static_cast<int>(q.active.size());
            const std::vector<double> rn = column_norms(p, Rres + t * blk, na, s);
            std::vector<int32_t> keep_slot;
            std::vector<double> next_rn, next_tol;
            for (int sl = 0; sl < na; ++sl) {
                const int r = q.active[sl];
                if (!std::isfinite(rn[sl])) fail(VSIE_E_NAN, "non-finite residual");
                relres[t][r] = rn[sl] / q.bn[r];
                worst_start = std::max(worst_start, relres[t][r]);
                if (relres[t][r] <= o.tol) continue;
                if (cnt[t].it[r] >= o.max_iter || (prec == VSIE_FP32 && cnt[t].outer[r] >= o.max_outer)) {
                    status[t] = VSIE_E_NOCONV;
                    continue;
                }
                double tl = o.tol * q.bn[r] / rn[sl];
                if (prec == VSIE_FP32) tl = std::max(tl, o.inner_tol);
                next[t].push_back(r);
                keep_slot.push_back(sl);
                next_rn.push_back(rn[sl]);
                next_tol.push_back(tl);
            }
            if (next[t].empty()) continue;
            double2 *cyc_res = Rres + t * blk;
            if (static_cast<int>(next[t].size()) != na) {  // compact the residual block
                to_device(act, keep_slot, s);
                bblas_gather(n, static_cast<int>(next[t].size()), act, Rres + t * blk, n, Xa + t * blk, s);
                cyc_res = Xa + t * blk;
            }
            for (int r : next[t]) cnt[t].outer[r]++;
            const int Ra = static_cast<int>(next[t].size());
            const int mb = multi_restart(n, Ra, o, nf);
            double2 *V = (q.have_first ? V2b : Vb) + t * region;
            cyc[t] = std::make_unique<BlockCycle>(p, f0 + t, prec, next[t], cyc_res, next_rn, next_tol, mb,
                                                  o.max_iter, xcol(t), ldx, cnt[t], s, V, Wb + t * blk,
                                                  q.have_first ? nullptr : &q.first,
                                                  q.have_first && q.first.k > 0 ? &q.first : nullptr,
                                                  Bb + t * bm_stride, Qb + t * qk_stride, false);
            cyc[t]->begin();
        }
        if (p->progress) {
            int nl = 0;
            for (int t = 0; t < nf; ++t) nl += cyc[t] != nullptr;
            std::fprintf(stderr, "[vsie] lockstep refinement step: %d of %d frequencies iterate, max FP64 relative "
                                 "residual %.3e\n", nl, nf, worst_start);
            std::fflush(stderr);
        }
        // block steps in lockstep; a cycle that stops is finished at once
        std::vector<int> done(nf, -1);
        for (int step = 1;; ++step) {
            std::vector<ProdItem> prod;
            for (int t = 0; t < nf; ++t)
                if (cyc[t] && done[t] < 0) {
                    if (cyc[t]->wants_product()) prod.push_back({f0 + t, cyc[t]->width(), cyc[t]->input(), cyc[t]->output()});
                    else done[t] = cyc[t]->finish();
                }
            if (prod.empty()) break;
            const auto t0 = std::chrono::steady_clock::now();
            const int launches = apply_items(p, prec, prod, s);
            double op_s = 0.0;
            if (p->progress) {
                VSIE_HIP(hipStreamSynchronize(s));
                op_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            }
            double worst = 0.0;
            for (const ProdItem &it : prod) {
                BlockCycle &c = *cyc[it.f - f0];
                c.after_product();
                worst = std::max(worst, c.worst());
            }
            if (p->progress) {
                std::fprintf(stderr, "[vsie] lockstep block step %d: %zu frequencies in %d multi-frequency "
                                     "product%s (%.3f s), max residual estimate %.3e of the cycle start\n",
                             step, prod.size(), launches, launches == 1 ? "" : "s", op_s, worst);
                std::fflush(stderr);
            }
        }
        for (int t : live) {
            Freq &q = F[t];
            if (!cyc[t]) {
                q.active.clear();
                continue;
            }
            q.have_first = true;
            for (int r : next[t]) q.xzero[r] = 0;
            if (done[t] == 0) {  // breakdown at the first step: no progress possible
                status[t] = VSIE_E_NOCONV;
                q.active.clear();
            } else {
                q.active = next[t];
            }
        }
    }
}

// Work buffers of solve_multi_batch: its own blocks and bases, every
// multi-frequency or single product it can issue, and the block cycles'
// shared buffers for every width up to R.
void plan_block_cycles(vsie_problem *p, int R, int nf, const std::function<int(int)> &steps, WsPlan &pl);

void plan_solve_multi(vsie_problem *p, int f0, int nf, vsie_precision prec, int R, const vsie_solve_opts &o,
                      WsPlan &pl) {
    const int64_t n = p->m.n;
    const size_t z = sizeof(double2), blk = z * static_cast<size_t>(n) * R;
    const int64_t region = multi_basis_cols(n, R, o, nf) * n;
    pl.need(p->V, z * static_cast<size_t>(region) * nf);
    pl.need(p->V2, z * static_cast<size_t>(region) * nf);
    for (Scratch *b : {&p->w, &p->xa, &p->axa, &p->rres}) pl.need(*b, blk * nf);
    pl.need(p->r, blk);
    pl.need(p->act2, sizeof(int32_t) * R);
    pl.need(p->npart, sizeof(double) * norm_chunks(n) * R);
    pl.need(p->nrm, sizeof(double) * R);
    for (int Ra = 1; Ra <= R; ++Ra)
        for (vsie_precision pr : {VSIE_FP64, prec}) {
            for (int len = 1; len <= nf; ++len) plan_multi(p, f0, len, pr, Ra, pl);
            for (int t = 0; t < nf; ++t) plan_op(p, f0 + t, pr, false, Ra, pl);
        }
    plan_block_cycles(p, R, nf, [&](int Ra) { return multi_restart(n, Ra, o, nf); }, pl);
}

// The work buffers of solve_batch (either path) for R right-hand sides: upper
// bounds over every cycle, live-column count and refinement step, from the
// same size rules the solver uses.  Block GMRES's Gram-Schmidt products run
// on rocBLAS, whose handle keeps device memory of its own.
void plan_solve(vsie_problem *p, int f, vsie_precision prec, bool adjoint, int R, const vsie_solve_opts &o,
                WsPlan &pl) {
    const int64_t n = p->m.n;
    const size_t z = sizeof(double2), nR = z * static_cast<size_t>(n) * R;
    const int nch = norm_chunks(n);
    pl.need(p->act2, sizeof(int32_t) * R);
    for (Scratch *b : {&p->r, &p->xa, &p->axa, &p->rres}) pl.need(*b, nR);
    pl.need(p->npart, sizeof(double) * nch * R);
    pl.need(p->nrm, sizeof(double) * R);
    for (int nl = 1; nl <= R; ++nl) {
        plan_op(p, f, VSIE_FP64, adjoint, nl, pl);
        if (prec == VSIE_FP32) plan_op(p, f, VSIE_FP32, adjoint, nl, pl);
    }
    if (!o.block) {
        const int m = gmres_restart(n, R, o);
        const size_t ns = R, hs = m + 2, cs = m + 2;  // recycled dimensions are at most m
        pl.need(p->V, nR * (m + 1));
        pl.need(p->V2, nR * (m + 1));
        pl.need(p->w, nR);
        pl.need(p->ax, nR);
        pl.need(p->h1, z * 2 * hs * ns + sizeof(double) * ns);
        pl.need(p->tc, z * cs * ns);
        pl.need(p->dpart, z * nch * (m + 1) * ns);
        pl.need(p->yv, z * cs * ns);
        pl.need(p->defP, z * cs * cs * ns);
        pl.need(p->defM, z * cs * cs * ns);
        pl.need(p->defB, z * static_cast<size_t>(m) * m * ns);
        for (Scratch *b : {&p->act, &p->live, &p->kc, &p->kd, &p->defk, &p->lslot}) pl.need(*b, sizeof(int32_t) * ns);
        return;
    }
    int64_t vcols = 0;
    for (int Ra = 1; Ra <= R; ++Ra)
        vcols = std::max<int64_t>(vcols, static_cast<int64_t>(Ra) * (block_restart(n, Ra, o) + 1));
    plan_block_cycles(p, R, 1, [&](int Ra) { return block_restart(n, Ra, o); }, pl);
    pl.need(p->V, z * static_cast<size_t>(n) * vcols);
    pl.need(p->V2, z * static_cast<size_t>(n) * vcols);
    pl.need(p->w, nR);
}

// The shared buffers of block cycles of every width up to R, steps(Ra) block
// steps per cycle of width Ra, and the deflation buffers of nf frequencies.
void plan_block_cycles(vsie_problem *p, int R, int nf, const std::function<int(int)> &steps, WsPlan &pl) {
    const int64_t n = p->m.n;
    const size_t z = sizeof(double2);
    int64_t kmax = 0;
    for (int Ra = 1; Ra <= R; ++Ra) {
        const int mb = steps(Ra);
        kmax = std::max<int64_t>(kmax, static_cast<int64_t>(Ra) * mb);
        pl.need(p->bh, z * static_cast<size_t>(mb + 1) * Ra * Ra);
        pl.need(p->bg, z * static_cast<size_t>(Ra) * Ra * (Ra <= kSmallChol ? 5 : 1));
        if (Ra <= kSmallChol) pl.need(p->bst, z * stage_len(static_cast<int64_t>(mb + 1) * Ra, Ra));
        pl.need(p->bsk, tall_bytes(Ra, Ra, n));
        for (int j = 0; j < mb; ++j) pl.need(p->bsk, tall_bytes(static_cast<int64_t>(j + 1) * Ra, Ra, n));
    }
    // a kept first cycle has at most kBlockRecycleMax columns, from at most R
    const int64_t kv = std::min(kmax, kBlockRecycleMax) + R;
    for (int Ra = 1; Ra <= R; ++Ra)
        for (int64_t k = 1; k <= kv; ++k) pl.need(p->bsk, tall_bytes(k, Ra, n));
    pl.need(p->brc, z * static_cast<size_t>(kv) * R);
    pl.need(p->ax, z * static_cast<size_t>(n) * R);
    pl.need(p->act, sizeof(int32_t) * R);
    const DeflateCaps dc = deflate_caps(R, steps);
    pl.need(p->bqk, dc.qk * nf);
    pl.need(p->bbm, dc.bm * nf);
    pl.need(p->bzt, dc.zt);
}

// Solver options with defaults, validated.
vsie_solve_opts solve_options(const vsie_solve_opts *opts) {
    vsie_solve_opts o{1e-10, 3000, 500, 1e-5, 20, 0, 0.0, 0, 0};
    if (opts) o = *opts;
    require(o.tol > 0 && o.max_iter >= 0 && o.restart >= 1 && o.restart <= 20000 && o.inner_tol > 0 &&
                o.inner_tol < 1 && o.max_outer >= 1 && (o.block == 0 || o.block == 1) && o.relax >= 0 &&
                o.relax < 1 && (o.progress == 0 || o.progress == 1) && o.krylov_gib >= 0 &&
                o.krylov_gib <= 4096,
            "invalid solver options");
    return o;
}

}  // namespace

// ---------------------------------------------------------------------------
// Work area of vsie_matvec_noalloc, for callers that cannot allocate device
// memory: a static device array, one copy per GPU, held until the process
// ends.  In host code `scratch` is only a stand-in for the device symbol, not
// a device address; each device's address comes from hipGetSymbolAddress
// (taken once per device, with that device current) and only that address is
// used.  Every work buffer of a product is fully written by the launches that
// read it, so nothing in the area needs clearing between calls; calls that
// overlap on one GPU share the area and race.
constexpr size_t kNoAllocBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};

void *noalloc_area(int device) {
    require(device >= 0 && device < kMaxDevices, "device index out of range");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void *q = nullptr;
        VSIE_HIP(hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)));
        require(q != nullptr && reinterpret_cast<uintptr_t>(q) % kWsAlign == 0, "static work area not addressable");
        g_noalloc_ptr[device] = q;
    }
    return g_noalloc_ptr[device];
}

// Pair-launch timing off for the duration of a call (its events would be
// created on demand).
struct ProfilerPause {
    PairProfiler &pr;
    bool was;
    explicit ProfilerPause(vsie_problem *p) : pr(p->prof), was(p->prof.on) { pr.on = false; }
    ~ProfilerPause() { pr.on = was; }
};

}  // namespace

// ---------------------------------------------------------------------------
// ABI

extern "C" {

vsie_status vsie_matvec_noalloc(vsie_problem *p, int32_t f, vsie_precision prec, int64_t nrhs, const double *x,
                                int64_t ldx, double *y, int64_t ldy, void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(prec == VSIE_FP64 || prec == VSIE_FP32, "unknown precision");
        require(nrhs >= 1 && nrhs <= 4096, "nrhs must be in [1, 4096]");
        check_vec(x, ldx, p->m.n, "x");
        check_vec(y, ldy, p->m.n, "y");
        int dev = -1;
        VSIE_HIP(hipGetDevice(&dev));
        require(dev == p->device, "the problem's device must be the current device");
        WsPlan pl;
        plan_op(p, f, prec, false, static_cast<int>(nrhs), pl);
        const size_t need = pl.total();
        if (need > kNoAllocBytes)
            fail(VSIE_E_WORKSPACE, "the product needs " + std::to_string(need) +
                                       " bytes of work buffers; the static work area holds " +
                                       std::to_string(kNoAllocBytes));
        void *area = noalloc_area(dev);
        ProfilerPause pause(p);
        WsScope ws(pl, area, kNoAllocBytes);
        apply_op(p, f, prec, false, static_cast<int>(nrhs), reinterpret_cast<const double2 *>(x), ldx,
                 reinterpret_cast<double2 *>(y), ldy, as_stream(stream));
    });
}

const char *vsie_last_error(void) { return g_last_error.c_str(); }

int64_t vsie_size(const vsie_problem *p) { return p ? p->m.n : 0; }

int64_t vsie_num_cells(const vsie_problem *p) { return p ? p->m.n_vol : 0; }

void vsie_destroy(vsie_problem *p) { delete p; }

vsie_status vsie_assemble(const vsie_geometry *geom, const double *vrho, const double *vc,
                          const double *k0, int32_t n_freq, void *stream, vsie_problem **out) {
    if (out) *out = nullptr;
    return guarded([&] {
        require(out != nullptr, "output handle pointer is NULL");
        validate_geometry(geom, vrho, vc);
        require(k0 != nullptr && n_freq >= 1, "need at least one wavenumber");
        for (int f = 0; f < n_freq; ++f)
            require(std::isfinite(k0[f]) && k0[f] > 0, "wavenumbers must be positive");
        std::unique_ptr<vsie_problem> p(new vsie_problem());
        VSIE_HIP(hipGetDevice(&p->device));
        hipStream_t s = as_stream(stream);
        const vsie_geometry &g = *geom;
        DeviceMesh &m = p->m;
        m.n_vol = g.n_vol;
        m.n_srf = g.n_srf;
        m.n = g.n_vol + g.n_srf;
        m.rho0 = g.rho0;
        m.c0 = g.c0;
        std::vector<double> px(m.n), py(m.n), pz(m.n);
        for (int64_t e = 0; e < g.n_vol; ++e) {
            px[e] = g.vx[e];
            py[e] = g.vy[e];
            pz[e] = g.vz[e];
        }
        for (int64_t q = 0; q < g.n_srf; ++q) {
            px[g.n_vol + q] = g.sx[q];
            py[g.n_vol + q] = g.sy[q];
            pz[g.n_vol + q] = g.sz[q];
        }
        m.px = p->upload(px.data(), m.n);
        m.py = p->upload(py.data(), m.n);
        m.pz = p->upload(pz.data(), m.n);
        m.vw = p->upload(g.vw, g.n_vol);
        m.vdom = p->upload(g.vdom, g.n_vol);
        m.vnb = g.vnb ? p->upload(g.vnb, 6 * g.n_vol) : nullptr;
        m.vga = g.vgrad_alpha ? p->upload(g.vgrad_alpha, 3 * g.n_vol) : nullptr;
        m.vgr = (g.vgrad_rho && !g.vgrad_alpha) ? p->upload(g.vgrad_rho, 3 * g.n_vol) : nullptr;
        m.vrho = p->upload(vrho, g.n_vol);
        m.vc = p->upload(vc, g.n_vol);
        m.snx = p->upload(g.snx, g.n_srf);
        m.sny = p->upload(g.sny, g.n_srf);
        m.snz = p->upload(g.snz, g.n_srf);
        m.sarea = p->upload(g.sarea, g.n_srf);
        m.siface = p->upload(g.siface, g.n_srf);
        m.scin = p->upload(g.scell_in, g.n_srf);
        m.scout = p->upload(g.scell_out, g.n_srf);
        m.vpx = p->alloc<double>(m.n);
        m.vpy = p->alloc<double>(m.n);
        m.vpz = p->alloc<double>(m.n);
        m.mass = p->alloc<double>(m.n);
        m.sp = p->alloc<double>(m.n * n_freq);
        m.diag = p->alloc<double2>(m.n * n_freq);
        // cell -> adjacent faces, for the density gradient through interface weights
        {
            std::vector<int32_t> off(g.n_vol + 1, 0), idx;
            for (int64_t q = 0; q < g.n_srf; ++q) {
                off[g.scell_in[q] + 1]++;
                if (g.scell_out[q] >= 0) off[g.scell_out[q] + 1]++;
            }
            for (int64_t e = 0; e < g.n_vol; ++e) off[e + 1] += off[e];
            idx.resize(off[g.n_vol]);
            std::vector<int32_t> fill(off.begin(), off.end() - 1);
            for (int64_t q = 0; q < g.n_srf; ++q) {
                idx[fill[g.scell_in[q]]++] = static_cast<int32_t>(q);
                if (g.scell_out[q] >= 0) idx[fill[g.scell_out[q]]++] = static_cast<int32_t>(q);
            }
            if (g.n_vol > 0) p->cf_off = p->upload(off.data(), g.n_vol + 1);
            if (!idx.empty()) p->cf_idx = p->upload(idx.data(), static_cast<int64_t>(idx.size()));
        }
        p->k0.assign(k0, k0 + n_freq);
        p->dense.assign(n_freq, vsie_problem::Dense{});
        p->d_k0 = p->upload(k0, n_freq);
        launch_weights(m, p->d_k0, n_freq, s);
        VSIE_HIP(hipStreamSynchronize(s));
        build_sources(p.get());
        *out = p.release();
    });
}

vsie_status vsie_set_materials(vsie_problem *p, const double *vrho_dev, const double *vc_dev,
                               void *stream) {
    return guarded([&] {
        require(p != nullptr, "problem handle is NULL");
        require(p->m.n_vol == 0 || (vrho_dev && vc_dev), "material arrays must not be NULL");
        hipStream_t s = as_stream(stream);
        if (p->m.n_vol > 0) {
            // validate a host copy first: rejected materials leave the problem
            // (materials, weights, sources) exactly as it was
            std::vector<double> hr(p->m.n_vol), hc(p->m.n_vol);
            VSIE_HIP(hipMemcpyAsync(hr.data(), vrho_dev, sizeof(double) * p->m.n_vol, hipMemcpyDeviceToHost, s));
            VSIE_HIP(hipMemcpyAsync(hc.data(), vc_dev, sizeof(double) * p->m.n_vol, hipMemcpyDeviceToHost, s));
            VSIE_HIP(hipStreamSynchronize(s));
            for (int64_t e = 0; e < p->m.n_vol; ++e)
                require(hr[e] > 0 && std::isfinite(hr[e]) && hc[e] > 0 && std::isfinite(hc[e]),
                        "density and sound speed must be positive at cell " + std::to_string(e));
            VSIE_HIP(hipMemcpyAsync(p->m.vrho, hr.data(), sizeof(double) * p->m.n_vol, hipMemcpyHostToDevice, s));
            VSIE_HIP(hipMemcpyAsync(p->m.vc, hc.data(), sizeof(double) * p->m.n_vol, hipMemcpyHostToDevice, s));
            VSIE_HIP(hipStreamSynchronize(s));
        }
        launch_weights(p->m, p->d_k0, static_cast<int>(p->k0.size()), s);
        VSIE_HIP(hipStreamSynchronize(s));
        const bool changed = build_sources(p);
        // assembled operators describe the old materials
        bool had_dense = false;
        for (auto &d : p->dense) {
            had_dense = had_dense || d.A != nullptr;
            d = vsie_problem::Dense{};
        }
        // captured operator graphs stay valid while the source lists, their
        // arrays and the tile flags are the same (the weights, the diagonal and
        // v' are rewritten in place)
        if (changed || had_dense) ++g_graph_epoch;
    });
}

vsie_status vsie_matvec(vsie_problem *p, int32_t f, vsie_precision prec, int64_t nrhs,
                        const double *x, int64_t ldx, double *y, int64_t ldy, void *workspace, size_t ws_bytes,
                        void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(prec == VSIE_FP64 || prec == VSIE_FP32, "unknown precision");
        require(nrhs >= 1 && nrhs <= 4096, "nrhs must be in [1, 4096]");
        check_vec(x, ldx, p->m.n, "x");
        check_vec(y, ldy, p->m.n, "y");
        WsPlan pl;
        if (workspace) plan_op(p, f, prec, false, static_cast<int>(nrhs), pl);
        WsScope ws(pl, workspace, ws_bytes);
        apply_op(p, f, prec, false, static_cast<int>(nrhs), reinterpret_cast<const double2 *>(x), ldx,
                 reinterpret_cast<double2 *>(y), ldy, as_stream(stream));
    });
}

vsie_status vsie_matvec_adjoint(vsie_problem *p, int32_t f, vsie_precision prec, int64_t nrhs,
                                const double *x, int64_t ldx, double *y, int64_t ldy,
                                void *workspace, size_t ws_bytes, void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(prec == VSIE_FP64 || prec == VSIE_FP32, "unknown precision");
        require(nrhs >= 1 && nrhs <= 4096, "nrhs must be in [1, 4096]");
        check_vec(x, ldx, p->m.n, "x");
        check_vec(y, ldy, p->m.n, "y");
        WsPlan pl;
        if (workspace) plan_op(p, f, prec, true, static_cast<int>(nrhs), pl);
        WsScope ws(pl, workspace, ws_bytes);
        apply_op(p, f, prec, true, static_cast<int>(nrhs), reinterpret_cast<const double2 *>(x), ldx,
                 reinterpret_cast<double2 *>(y), ldy, as_stream(stream));
    });
}

vsie_status vsie_matvec_multi(vsie_problem *p, int32_t f0, int32_t nf, vsie_precision prec, int64_t nrhs,
                              const double *x, int64_t ldx, double *y, int64_t ldy, void *workspace,
                              size_t ws_bytes, void *stream) {
    return guarded([&] {
        require(p != nullptr, "problem handle is NULL");
        require(nf >= 1 && f0 >= 0 && static_cast<int64_t>(f0) + nf <= static_cast<int64_t>(p->k0.size()),
                "frequency range out of bounds");
        require(prec == VSIE_FP64 || prec == VSIE_FP32, "unknown precision");
        require(nrhs >= 1 && nrhs <= 4096, "nrhs must be in [1, 4096]");
        check_vec(x, ldx, p->m.n, "x");
        check_vec(y, ldy, p->m.n, "y");
        WsPlan pl;
        if (workspace) plan_multi(p, f0, nf, prec, static_cast<int>(nrhs), pl);
        WsScope ws(pl, workspace, ws_bytes);
        hipStream_t s = as_stream(stream);
        const double2 *xv = reinterpret_cast<const double2 *>(x);
        double2 *yv = reinterpret_cast<double2 *>(y);
        const int R = static_cast<int>(nrhs);
        bool dense = false;
        for (int t = 0; t < nf; ++t) dense = dense || p->dense[f0 + t].A != nullptr;
        if (use_mfma(p, prec, R) && !dense) {
            apply_forward_mfma(p, f0, nf, R, xv, ldx, nrhs * ldx, yv, ldy, nrhs * ldy, s);
            return;
        }
        if (use_mfma64(p, prec, R)) {
            apply_forward_mfma64(p, f0, nf, R, xv, ldx, nrhs * ldx, yv, ldy, nrhs * ldy, s);
            return;
        }
        for (int t = 0; t < nf; ++t)
            apply_op(p, f0 + t, prec, false, R, xv + t * nrhs * ldx, ldx, yv + t * nrhs * ldy, ldy, s);
    });
}

vsie_status vsie_get_tuning(const vsie_problem *p, vsie_tuning *out) {
    return guarded([&] {
        require(p != nullptr && out != nullptr, "NULL argument");
        *out = p->tune;
    });
}

vsie_status vsie_set_tuning(vsie_problem *p, const vsie_tuning *t) {
    return guarded([&] {
        require(p != nullptr && t != nullptr, "NULL argument");
        check_tuning(*t);
        p->tune = *t;
        ++g_graph_epoch;
    });
}

vsie_status vsie_autotune(vsie_problem *p, int32_t f, int64_t nrhs, vsie_tuning *best, void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(nrhs >= 1 && nrhs <= 4096, "nrhs must be in [1, 4096]");
        hipStream_t s = as_stream(stream);
        const int64_t n = p->m.n;
        const int R = static_cast<int>(nrhs);
        struct Buf {
            void *d = nullptr;
            ~Buf() {
                if (d) (void)hipFree(d);
            }
        } X, Y;
        VSIE_HIP(hipMalloc(&X.d, sizeof(double2) * static_cast<size_t>(n) * R));
        VSIE_HIP(hipMalloc(&Y.d, sizeof(double2) * static_cast<size_t>(n) * R));
        double2 *xd = static_cast<double2 *>(X.d), *yd = static_cast<double2 *>(Y.d);
        // inputs: plane waves along a spread of directions
        for (int r = 0; r < R; ++r) {
            const double t = (r + 0.5) / R, z = 1.0 - 2.0 * t, rho = std::sqrt(std::max(0.0, 1.0 - z * z));
            const double ph = 2.399963229728653 * r;
            launch_plane_wave(n, p->m.px, p->m.py, p->m.pz, p->k0[f], rho * std::cos(ph), rho * std::sin(ph), z,
                              xd + static_cast<int64_t>(r) * n, s);
        }
        std::vector<vsie_tuning> cand;
        const vsie_tuning base = p->tune;
        for (int64_t tw : {16384, 32768, 65536}) {
            vsie_tuning t = base;
            t.mfma_min_rhs = 0;
            t.vec_target_waves = tw;
            cand.push_back(t);
        }
        if (R >= 8)
            for (auto tn : {std::make_pair(2, 1), std::make_pair(4, 1), std::make_pair(2, 2)})
                for (int ipw : {8, 16, 32}) {
                    vsie_tuning t = base;
                    t.mfma_min_rhs = std::min(8, R);
                    t.mfma_tg = tn.first;
                    t.mfma_nb = tn.second;
                    t.items_per_wave = ipw;
                    cand.push_back(t);
                }
        hipEvent_t e0, e1;
        VSIE_HIP(hipEventCreate(&e0));
        VSIE_HIP(hipEventCreate(&e1));
        double best_ms = 1e300;
        vsie_tuning pick = base;
        const bool prof_on = p->prof.on;
        p->prof.on = false;
        try {
            for (const auto &t : cand) {
                p->tune = t;
                auto run = [&] {
                    if (use_mfma(p, VSIE_FP32, R)) apply_forward_mfma(p, f, 1, R, xd, n, 0, yd, n, 0, s);
                    else apply_forward(p, f, VSIE_FP32, R, xd, n, yd, n, s);
                };
                run();  // warm-up (buffers, code objects)
                VSIE_HIP(hipEventRecord(e0, s));
                run();
                run();
                VSIE_HIP(hipEventRecord(e1, s));
                VSIE_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                VSIE_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best_ms) {
                    best_ms = ms;
                    pick = t;
                }
            }
        } catch (...) {
            p->tune = base;
            p->prof.on = prof_on;
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        p->prof.on = prof_on;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        // the vector kernel won: keep the matrix cores for wider blocks only
        if (pick.mfma_min_rhs == 0 && base.mfma_min_rhs > 0) pick.mfma_min_rhs = std::max(base.mfma_min_rhs, R + 1);
        p->tune = pick;
        ++g_graph_epoch;
        if (best) *best = pick;
    });
}

vsie_status vsie_solve(vsie_problem *p, int32_t f, vsie_precision prec, int32_t adjoint,
                       int64_t nrhs, const double *b, int64_t ldb, double *x, int64_t ldx,
                       const vsie_solve_opts *opts, vsie_solve_info *info, void *workspace, size_t ws_bytes,
                       void *stream) {
    if (info) *info = vsie_solve_info{0, 0, 0, 0, 0.0};
    vsie_status result = VSIE_OK;
    const vsie_status st = guarded([&] {
        check_problem(p, f);
        require(prec == VSIE_FP64 || prec == VSIE_FP32, "unknown precision");
        require(adjoint == 0 || adjoint == 1, "adjoint must be 0 or 1");
        require(nrhs >= 1 && nrhs <= 4096, "nrhs must be in [1, 4096]");
        check_vec(b, ldb, p->m.n, "b");
        check_vec(x, ldx, p->m.n, "x");
        const vsie_solve_opts o = solve_options(opts);
        const int R = static_cast<int>(nrhs);
        WsPlan pl;
        if (workspace) plan_solve(p, f, prec, adjoint != 0, R, o, pl);
        WsScope ws(pl, workspace, ws_bytes);
        p->progress = o.progress;
        hipStream_t s = as_stream(stream);
        SolveCounters cnt(R);
        std::vector<double> rr;
        result = solve_batch(p, f, prec, adjoint != 0, R, reinterpret_cast<const double2 *>(b), ldb,
                             reinterpret_cast<double2 *>(x), ldx, o, cnt, rr, s);
        VSIE_HIP(hipStreamSynchronize(s));
        vsie_solve_info total{0, 0, 0, 0, 0.0};
        for (int r = 0; r < R; ++r) {
            total.iterations += cnt.it[r];
            total.matvecs_fp64 += cnt.mv64[r];
            total.matvecs_fp32 += cnt.mv32[r];
            total.outer_steps = std::max(total.outer_steps, cnt.outer[r]);
            total.rel_residual = std::max(total.rel_residual, rr[r]);
        }
        if (info) *info = total;
        if (result == VSIE_E_NOCONV) g_last_error = "GMRES did not reach the tolerance";
    });
    // an error part-way leaves no queued work behind the return
    if (st != VSIE_OK && p) (void)hipStreamSynchronize(as_stream(stream));
    return st != VSIE_OK ? st : result;
}

vsie_status vsie_solve_multi(vsie_problem *p, int32_t f0, int32_t nf, vsie_precision prec, int64_t nrhs,
                             const double *b, int64_t ldb, double *x, int64_t ldx, const vsie_solve_opts *opts,
                             vsie_solve_info *info, void *workspace, size_t ws_bytes, void *stream) {
    if (info && nf > 0)
        for (int t = 0; t < nf; ++t) info[t] = vsie_solve_info{0, 0, 0, 0, 0.0};
    vsie_status result = VSIE_OK;
    const vsie_status st = guarded([&] {
        require(p != nullptr, "problem handle is NULL");
        require(nf >= 1 && f0 >= 0 && static_cast<int64_t>(f0) + nf <= static_cast<int64_t>(p->k0.size()),
                "frequency range out of bounds");
        require(prec == VSIE_FP64 || prec == VSIE_FP32, "unknown precision");
        require(nrhs >= 1 && nrhs <= 4096, "nrhs must be in [1, 4096]");
        check_vec(b, ldb, p->m.n, "b");
        check_vec(x, ldx, p->m.n, "x");
        const vsie_solve_opts o = solve_options(opts);
        const int R = static_cast<int>(nrhs);
        WsPlan pl;
        if (workspace) plan_solve_multi(p, f0, nf, prec, R, o, pl);
        WsScope ws(pl, workspace, ws_bytes);
        p->progress = o.progress;
        hipStream_t s = as_stream(stream);
        std::vector<SolveCounters> cnt(nf, SolveCounters(R));
        std::vector<std::vector<double>> rr(nf);
        std::vector<vsie_status> fs(nf, VSIE_OK);
        solve_multi_batch(p, f0, nf, prec, R, reinterpret_cast<const double2 *>(b), ldb,
                          reinterpret_cast<double2 *>(x), ldx, o, cnt, rr, fs, s);
        VSIE_HIP(hipStreamSynchronize(s));
        for (int t = 0; t < nf; ++t) {
            vsie_solve_info tot{0, 0, 0, 0, 0.0};
            for (int r = 0; r < R; ++r) {
                tot.iterations += cnt[t].it[r];
                tot.matvecs_fp64 += cnt[t].mv64[r];
                tot.matvecs_fp32 += cnt[t].mv32[r];
                tot.outer_steps = std::max(tot.outer_steps, cnt[t].outer[r]);
                tot.rel_residual = std::max(tot.rel_residual, rr[t][r]);
            }
            if (info) info[t] = tot;
            if (fs[t] != VSIE_OK) result = fs[t];
        }
        if (result == VSIE_E_NOCONV) g_last_error = "GMRES did not reach the tolerance at every frequency";
    });
    if (st != VSIE_OK && p) (void)hipStreamSynchronize(as_stream(stream));
    return st != VSIE_OK ? st : result;
}

vsie_status vsie_workspace_size(vsie_problem *p, vsie_op op, int32_t f, int32_t nf, vsie_precision prec,
                                int64_t nrhs, const vsie_solve_opts *opts, size_t *bytes) {
    if (bytes) *bytes = 0;
    return guarded([&] {
        require(bytes != nullptr, "bytes is NULL");
        check_problem(p, f);
        require(prec == VSIE_FP64 || prec == VSIE_FP32, "unknown precision");
        require(nrhs >= 1 && nrhs <= 4096, "nrhs must be in [1, 4096]");
        if (op == VSIE_OP_MATVEC_MULTI || op == VSIE_OP_SOLVE_MULTI)
            require(nf >= 1 && static_cast<int64_t>(f) + nf <= static_cast<int64_t>(p->k0.size()),
                    "frequency range out of bounds");
        else
            require(nf == 1, "nf must be 1 except for the multi-frequency calls");
        const int R = static_cast<int>(nrhs);
        WsPlan pl;
        switch (op) {
        case VSIE_OP_MATVEC: plan_op(p, f, prec, false, R, pl); break;
        case VSIE_OP_MATVEC_ADJOINT: plan_op(p, f, prec, true, R, pl); break;
        case VSIE_OP_MATVEC_MULTI: plan_multi(p, f, nf, prec, R, pl); break;
        case VSIE_OP_SOLVE:
        case VSIE_OP_SOLVE_ADJOINT: plan_solve(p, f, prec, op == VSIE_OP_SOLVE_ADJOINT, R, solve_options(opts), pl); break;
        case VSIE_OP_SOLVE_MULTI: plan_solve_multi(p, f, nf, prec, R, solve_options(opts), pl); break;
        default: fail(VSIE_E_INVALID, "unknown operation");
        }
        *bytes = pl.total();
    });
}

vsie_status vsie_plane_wave(vsie_problem *p, int32_t f, int64_t ndir, const double *dirs, double *b,
                            int64_t ldb, void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(ndir >= 1 && dirs != nullptr, "need at least one direction");
        check_vec(b, ldb, p->m.n, "b");
        for (int64_t d = 0; d < ndir; ++d) {
            const double *u = dirs + 3 * d;
            const double nn = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            require(std::fabs(nn - 1.0) <= 1e-12, "direction not of unit length");
            launch_plane_wave(p->m.n, p->m.px, p->m.py, p->m.pz, p->k0[f], u[0], u[1], u[2],
                              reinterpret_cast<double2 *>(b) + d * ldb, as_stream(stream));
        }
    });
}

vsie_status vsie_field(vsie_problem *p, int32_t f, vsie_precision prec, int64_t n_t, const double *tx,
                       const double *ty, const double *tz, int64_t nrhs, const double *x, int64_t ldx,
                       double *out, int64_t ldo, void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(prec == VSIE_FP64 || prec == VSIE_FP32, "unknown precision");
        require(n_t >= 1 && tx && ty && tz, "need target points");
        require(nrhs >= 1 && nrhs <= 4096, "nrhs must be in [1, 4096]");
        check_vec(x, ldx, p->m.n, "x");
        check_vec(out, ldo, n_t, "out");
        hipStream_t s = as_stream(stream);
        const int R = static_cast<int>(nrhs);
        const int64_t n = p->m.n;
        int64_t chG, chF;
        int ncG, ncF;
        choose_chunks(n_t, p->G.count, p->tune.vec_target_waves, chG, ncG);
        choose_chunks(n_t, p->F.count, p->tune.vec_target_waves, chF, ncF);
        double2 *part = static_cast<double2 *>(
            p->partial.get(sizeof(double2) * static_cast<size_t>(std::max(1, ncG + ncF)) * R * n_t));
        void *qG = p->chargeG.get(csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->G.count)) * R);
        void *qF = p->chargeF.get(csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->F.count)) * R);
        const double *spf = p->m.sp + static_cast<int64_t>(f) * n;
        const double2 *xv = reinterpret_cast<const double2 *>(x);
        launch_pack_charges(kClassG, prec, p->G, spf, R, xv, ldx, false, qG, s);
        launch_pack_charges(kClassF, prec, p->F, spf, R, xv, ldx, false, qF, s);
        if (ncG > 0) {
            PairJob J{PAIR_FWD_G, prec, n_t, tx, ty, tz, {}, p->G.count, p->G.x, p->G.y, p->G.z,
                      {}, qG, p->G.count, R, chG, ncG, p->k0[f], part, static_cast<int64_t>(R) * n_t};
            launch_pairs(J, s, &p->prof);
        }
        if (ncF > 0) {
            PairJob J{PAIR_FWD_F, prec, n_t, tx, ty, tz, {}, p->F.count, p->F.x, p->F.y, p->F.z,
                      {p->F.vx, p->F.vy, p->F.vz}, qF, p->F.count, R,
                      chF, ncF, p->k0[f], part + static_cast<int64_t>(ncG) * R * n_t,
                      static_cast<int64_t>(R) * n_t};
            launch_pairs(J, s, &p->prof);
        }
        launch_reduce_partials(n_t, R, ncG + ncF, part, nullptr, false, nullptr, 0,
                               reinterpret_cast<double2 *>(out), ldo, nullptr, s);
    });
}

vsie_status vsie_far_field(vsie_problem *p, int32_t f, vsie_precision prec, int64_t n_d, const double *dx,
                           const double *dy, const double *dz, int64_t nrhs, const double *x, int64_t ldx,
                           double *out, int64_t ldo, void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(prec == VSIE_FP64 || prec == VSIE_FP32, "unknown precision");
        require(n_d >= 1 && dx && dy && dz, "need directions");
        require(nrhs >= 1 && nrhs <= 4096, "nrhs must be in [1, 4096]");
        check_vec(x, ldx, p->m.n, "x");
        check_vec(out, ldo, n_d, "out");
        hipStream_t s = as_stream(stream);
        const int R = static_cast<int>(nrhs);
        const int64_t n = p->m.n;
        int64_t chG, chF;
        int ncG, ncF;
        const int64_t lanes = (n_d + far_field_lanes(R) - 1) / far_field_lanes(R);
        choose_chunks(lanes, p->G.count, p->tune.vec_target_waves, chG, ncG);
        choose_chunks(lanes, p->F.count, p->tune.vec_target_waves, chF, ncF);
        double2 *part = static_cast<double2 *>(
            p->partial.get(sizeof(double2) * static_cast<size_t>(std::max(1, ncG + ncF)) * R * n_d));
        void *qG = p->chargeG.get(csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->G.count)) * R);
        void *qF = p->chargeF.get(csize(prec) * static_cast<size_t>(std::max<int64_t>(1, p->F.count)) * R);
        const double *spf = p->m.sp + static_cast<int64_t>(f) * n;
        launch_pack_both(prec, p->G, p->F, spf, R, reinterpret_cast<const double2 *>(x), ldx, false, qG, qF, s);
        if (ncG > 0) {
            FarJob J{kClassG, prec, n_d, dx, dy, dz, p->G.count, p->G.pk, nullptr, qG, p->G.count,
                     R, chG, ncG, p->k0[f], part, static_cast<int64_t>(R) * n_d};
            launch_far_field(J, s, &p->prof);
        }
        if (ncF > 0) {
            FarJob J{kClassF, prec, n_d, dx, dy, dz, p->F.count, p->F.pk, p->F.pv, qF, p->F.count, R, chF, ncF,
                     p->k0[f],
                     part + static_cast<int64_t>(ncG) * R * n_d, static_cast<int64_t>(R) * n_d};
            launch_far_field(J, s, &p->prof);
        }
        launch_reduce_partials(n_d, R, ncG + ncF, part, nullptr, false, nullptr, 0,
                               reinterpret_cast<double2 *>(out), ldo, nullptr, s);
    });
}

vsie_status vsie_source_sums(vsie_problem *p, int32_t f, int64_t n_t, const double *tx,
                             const double *ty, const double *tz, int64_t nrhs, const double *lam,
                             int64_t ldl, double *z, int64_t ldz, double *Z, int64_t ldZ,
                             void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(nrhs >= 1 && nrhs <= 4096, "nrhs must be in [1, 4096]");
        const int64_t n = p->m.n;
        const bool colloc = tx == nullptr;
        if (colloc) require(n_t == n && ty == nullptr && tz == nullptr, "collocation targets need n_t == n");
        else require(n_t >= 1 && ty && tz, "need target points");
        check_vec(lam, ldl, n_t, "lam");
        check_vec(z, ldz, n, "z");
        check_vec(Z, ldZ, n, "Z");
        hipStream_t s = as_stream(stream);
        const int R = static_cast<int>(nrhs);
        void *q = p->chargeAll.get(sizeof(double2) * static_cast<size_t>(n_t) * R);
        launch_pack_plain(VSIE_FP64, n_t, R, reinterpret_cast<const double2 *>(lam), ldl, true, q, s);
        int64_t ch;
        int nc;
        choose_chunks(n, n_t, p->tune.vec_target_waves, ch, nc);
        double2 *part = static_cast<double2 *>(
            p->sums_part.get(sizeof(double2) * static_cast<size_t>(nc) * R * 4 * n));
        PairJob J{PAIR_SUMS, VSIE_FP64, n, p->m.px, p->m.py, p->m.pz, {}, n_t,
                  colloc ? p->m.px : tx, colloc ? p->m.py : ty, colloc ? p->m.pz : tz, {}, q, n_t, R,
                  ch, nc, p->k0[f], part, static_cast<int64_t>(R) * 4 * n,
                  colloc ? SELF_IDENT : SELF_NONE, nullptr};
        launch_pairs(J, s, &p->prof);
        launch_sums_reduce(n, R, nc, part, reinterpret_cast<double2 *>(z), ldz,
                           reinterpret_cast<double2 *>(Z), ldZ, s);
    });
}

vsie_status vsie_plane_wave_at(vsie_problem *p, int32_t f, int64_t ndir, const double *dirs,
                               int64_t n_t, const double *tx, const double *ty, const double *tz,
                               double *out, int64_t ldo, void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(ndir >= 1 && dirs != nullptr, "need at least one direction");
        require(n_t >= 1 && tx && ty && tz, "need target points");
        check_vec(out, ldo, n_t, "out");
        for (int64_t d = 0; d < ndir; ++d) {
            const double *u = dirs + 3 * d;
            const double nn = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            require(std::fabs(nn - 1.0) <= 1e-12, "direction not of unit length");
            launch_plane_wave_at(n_t, tx, ty, tz, p->k0[f], u[0], u[1], u[2],
                                 reinterpret_cast<double2 *>(out) + d * ldo, as_stream(stream));
        }
    });
}

vsie_status vsie_adjoint_rhs(vsie_problem *p, int32_t f, int64_t nrhs, const double *zR, int64_t ldz,
                             const double *ZR, int64_t ldZ, double *out, int64_t ldo, void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(nrhs >= 1, "nrhs must be >= 1");
        check_vec(zR, ldz, p->m.n, "zR");
        check_vec(ZR, ldZ, p->m.n, "ZR");
        check_vec(out, ldo, p->m.n, "out");
        launch_adjoint_rhs(p->m, f, static_cast<int>(nrhs), reinterpret_cast<const double2 *>(zR), ldz,
                           reinterpret_cast<const double2 *>(ZR), ldZ, reinterpret_cast<double2 *>(out),
                           ldo, as_stream(stream));
    });
}

vsie_status vsie_param_gradient(vsie_problem *p, int32_t f, int64_t nrhs, const double *P, int64_t ldp,
                                const double *lam, int64_t ldl, const double *z, int64_t ldz,
                                const double *Z, int64_t ldZ, const double *zR, int64_t ldzr,
                                const double *ZR, int64_t ldZr, double *grad_c, double *grad_rho,
                                void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(nrhs >= 1, "nrhs must be >= 1");
        const int64_t n = p->m.n;
        check_vec(P, ldp, n, "p");
        check_vec(lam, ldl, n, "lam");
        check_vec(z, ldz, n, "z");
        check_vec(Z, ldZ, n, "Z");
        check_vec(zR, ldzr, n, "zR");
        check_vec(ZR, ldZr, n, "ZR");
        require(p->m.n_vol == 0 || (grad_c && grad_rho), "gradient outputs must not be NULL");
        double *work = static_cast<double *>(p->grad_work.get(sizeof(double) * 5 * static_cast<size_t>(n)));
        auto c2 = [](const double *v) { return reinterpret_cast<const double2 *>(v); };
        launch_param_gradient(p->m, p->cf_off, p->cf_idx, p->k0[f], static_cast<int>(nrhs), c2(P), ldp,
                              c2(lam), ldl, c2(z), ldz, c2(Z), ldZ, c2(zR), ldzr, c2(ZR), ldZr, work,
                              grad_c, grad_rho, as_stream(stream));
    });
}

vsie_status vsie_assemble_dense(vsie_problem *p, int32_t f, void *dense, int64_t ld, void *stream) {
    return guarded([&] {
        check_problem(p, f);
        require(dense != nullptr, "dense matrix memory is NULL");
        require(ld >= p->m.n, "leading dimension smaller than n");
        require(p->m.n <= INT32_MAX && ld <= INT32_MAX, "dense operator too large for the GEMM");
        hipStream_t s = as_stream(stream);
        const double *vp[3] = {p->m.vpx, p->m.vpy, p->m.vpz};
        launch_assemble_dense(p->m.n, p->m.px, p->m.py, p->m.pz, p->m.sp + static_cast<int64_t>(f) * p->m.n,
                              vp[0], vp[1], vp[2], p->k0[f], static_cast<float *>(dense), ld, s);
        p->dense[f] = vsie_problem::Dense{static_cast<float *>(dense), ld};
        ++g_graph_epoch;
    });
}

vsie_status vsie_release_dense(vsie_problem *p, int32_t f) {
    return guarded([&] {
        check_problem(p, f);
        p->dense[f] = vsie_problem::Dense{};
        ++g_graph_epoch;
    });
}

vsie_status vsie_profile(vsie_problem *p, int32_t enable) {
    return guarded([&] {
        require(p != nullptr, "problem handle is NULL");
        if (enable) {
            VSIE_HIP(hipDeviceSynchronize());
            for (auto &r : p->prof.recs) {
                p->prof.pool.push_back(r.a);
                p->prof.pool.push_back(r.b);
            }
            p->prof.recs.clear();
        }
        p->prof.on = enable != 0;
    });
}

vsie_status vsie_profile_read(vsie_problem *p, int32_t kind, vsie_kernel_stats *out) {
    return guarded([&] {
        require(p != nullptr && out != nullptr, "NULL argument");
        require(kind >= 0 && kind < 23, "kernel kind out of range");
        vsie_kernel_stats st{0, 0.0, 0.0, 0.0};
        for (auto &r : p->prof.recs) {
            if (r.kind != kind) continue;
            VSIE_HIP(hipEventSynchronize(r.b));
            float ms = 0.f;
            VSIE_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            st.launches += 1;
            st.ms += ms;
            st.pairs += r.pairs;
            st.rhs_pairs += r.rhs_pairs;
        }
        *out = st;
    });
}

}  // extern "C"
