// Internal declarations shared by the HIP translation units of libvsie.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/vsie.h"

namespace vsie {

constexpr int kBlock = 256;          // threads per workgroup of the pair kernels (4 wave64)
constexpr int kMaxRhsPerLaunch = 16; // right-hand sides one pair-kernel launch accumulates

// Error raised inside the library and turned into a vsie_status at the ABI.
struct Error {
    vsie_status code;
    std::string msg;
};

[[noreturn]] void fail(vsie_status code, const std::string &msg);
void check_hip(hipError_t e, const char *what);
#define VSIE_HIP(call) ::vsie::check_hip((call), #call)

// Source classes of the pair sum.  A volume cell with both a single-layer
// weight and a grad-alpha weight appears in both lists.
//   G: contribution  exp(i k r)/r * u_j,                    u_j = -s'_j x_j
//   F: contribution  exp(i k r)/r * q_ij (i k r - 1) x_j,    q_ij = (x_i - y_j).v'_j / r^2
// with s' = s / (4 pi) and v' = v / (4 pi).
enum SrcClass { kClassG = 0, kClassF = 1 };

// Device buffers of a problem.  Everything is in canonical unknown order
// unless marked "class order".
struct DeviceMesh {
    int64_t n_vol = 0, n_srf = 0, n = 0;
    double rho0 = 1, c0 = 1;
    // collocation points (all n), FP64 and FP32 copies
    double *px = nullptr, *py = nullptr, *pz = nullptr;
    // volume data
    double *vw = nullptr;
    int32_t *vdom = nullptr, *vnb = nullptr;
    double *vga = nullptr;  // optional explicit grad alpha (3 n_vol, xyz interleaved)
    double *vgr = nullptr;  // optional analytic grad rho (3 n_vol, xyz interleaved)
    double *vrho = nullptr, *vc = nullptr;
    // surface data
    double *snx = nullptr, *sny = nullptr, *snz = nullptr, *sarea = nullptr;
    int32_t *siface = nullptr, *scin = nullptr, *scout = nullptr;
    // frequency independent weights: v' (3 x n SoA), mass function m (n)
    double *vpx = nullptr, *vpy = nullptr, *vpz = nullptr, *mass = nullptr;
    // per frequency: s' (n_freq x n), diagonal m - D (n_freq x n complex)
    double *sp = nullptr;
    double2 *diag = nullptr;
};

// Packed sources of one class in class order.
struct SourceSet {
    int64_t count = 0;
    int32_t *idx = nullptr;                 // canonical index of each class entry
    double *x = nullptr, *y = nullptr, *z = nullptr;    // FP64 centroids
    double *vx = nullptr, *vy = nullptr, *vz = nullptr; // v' (F class only)
    // matrix-core layout: (x, y, z, 0) and (v'x, v'y, v'z, 0) per source, then
    // kMfmaPad entries far from every point with v' = 0
    double4 *pk = nullptr, *pv = nullptr;
};
constexpr int kMfmaPad = 8;

// One pair-sum pass (pair_kernels.hip).  Thread points t (n_t) each sum over
// a chunk of streamed points s (n_s); out receives one FP64 partial per
// (chunk, right-hand side, component, thread point):
//   out[c * chunk_stride + (r * ncomp + comp) * n_t + i],  ncomp = 4 for SUMS, else 1.
enum PairMode { PAIR_FWD_G = 0, PAIR_FWD_F = 1, PAIR_ADJ_F = 2, PAIR_SUMS = 3 };
// Which streamed points can coincide with a thread point (the r = 0 pair that
// contributes zero):
//   SELF_NONE        unknown (arbitrary targets): every pair is checked
//   SELF_IDENT       thread and streamed points are the same list
//   SELF_STREAM_IDX  thread points are the collocation points in canonical
//                    order; streamed point j is canonical point self_idx[j]
//                    (self_idx increasing)
//   SELF_THREAD_IDX  streamed points are the collocation points; thread point
//                    t is canonical point self_idx[t] (self_idx increasing)
//   SELF_DISJOINT    no streamed point is a thread point: nothing is masked
enum SelfMode { SELF_NONE = 0, SELF_IDENT = 1, SELF_STREAM_IDX = 2, SELF_THREAD_IDX = 3, SELF_DISJOINT = 4 };
struct PairJob {
    int mode;
    vsie_precision prec;
    int64_t n_t;
    const double *tx, *ty, *tz;
    const double *tv[3];      // ADJ_F: v' of thread points
    int64_t n_s;
    const double *sx, *sy, *sz;
    const double *sv[3];      // FWD_F: v' of streamed points
    const void *charge;       // complex charges (double2 or float2), charge[r * ldq + j]
    int64_t ldq;
    int nrhs;
    int64_t chunk;            // streamed points per chunk
    int n_chunks;             // ceil(n_s / chunk)
    double k;
    double2 *out;
    int64_t chunk_stride;
    int self_mode = SELF_NONE;
    const int32_t *self_idx = nullptr;
};
// Optional timing of pair launches (one event pair per launch).
struct PairProfiler {
    bool on = false;
    struct Rec {
        hipEvent_t a, b;
        int kind;
        double pairs, rhs_pairs;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};
void launch_pairs(const PairJob &J, hipStream_t s, PairProfiler *prof = nullptr);
hipEvent_t prof_take_event(PairProfiler *prof);

// Far-field pattern of one source class (far_field.hip): n_d unit directions
// d, sources with the packed charges of the forward product (class G: u_j =
// -s'_j x_j; class F: x_j, with v'), one FP64 partial per (chunk, right-hand
// side, direction) of
//   G: -sum_j exp(-i k d.y_j) u_j,   F: -sum_j exp(-i k d.y_j) i k (d.v'_j) x_j
// at out[c * chunk_stride + r * n_d + t].  Profiler kinds 14 + 2 cls + (FP32).
struct FarJob {
    int cls;
    vsie_precision prec;
    int64_t n_d;
    const double *dx, *dy, *dz;
    int64_t n_s;
    const double4 *pk, *pv;   // SourceSet::pk, pv (pv for class F)
    const void *charge;       // complex charges (double2 or float2), charge[r * ldq + j]
    int64_t ldq;
    int nrhs;
    int64_t chunk;            // sources per chunk
    int n_chunks;             // ceil(n_s / chunk)
    double k;
    double2 *out;
    int64_t chunk_stride;
};
void launch_far_field(const FarJob &J, hipStream_t s, PairProfiler *prof = nullptr);
// Directions one lane of the far-field kernel evaluates for nrhs right-hand
// sides (the launch needs ceil(n_d / that) lanes per source chunk).
int far_field_lanes(int nrhs);

// FP32 forward pair sums of one source class on the matrix cores
// (mfma_kernels.hip), for nf frequencies and a block of right-hand sides in
// one launch.  Targets are the n_t collocation points.  Charges
// are source-major, ncol (a multiple of 16 nb) columns per source,
// q[fl * ldq_f + j * ncol + col], with kMfmaPad zero rows after n_s; chunk
// is a multiple of 4.  Output, for
// chunk c, column col < nrhs and target i:
//   out[fl * out_fstride + (part0 + c) * nrhs * n_t + col * n_t + i].
// tg: 16-target groups per wave (2 or 4); nb: 16-column blocks per item (1 or 2);
// grid: workgroups (a multiple of 8; 0 = one item per wave).
struct MfmaJob {
    int cls;
    int64_t n_t;
    const double *tx, *ty, *tz;
    int64_t n_s;
    const double4 *pk, *pv;       // SourceSet::pk, pv
    const float2 *q;
    int64_t ldq_f;                // >= (n_s + kMfmaPad) ncol
    int ncol, nrhs;
    const double *kf;  // device array: k of each local frequency
    int nf;
    int64_t chunk;
    int n_chunks;
    double2 *out;
    int64_t out_fstride;
    int part0;
    int tg, nb, grid;
    bool m3;  // three real matrix-core products per complex product instead of four
};
void launch_mfma_forward(const MfmaJob &J, hipStream_t s, PairProfiler *prof);
// The same product in FP64 on the FP64 matrix cores: FP64 kernel values and
// charges (double2, q[fl * ldq_f + j * ncol + col]), FP64 accumulation, two
// 16-target groups per wave, nb in {1, 2, 4} 16-column blocks per item.
struct Mfma64Job {
    int cls;
    int64_t n_t;
    const double *tx, *ty, *tz;
    int64_t n_s;
    const double4 *pk, *pv;
    const double2 *q;
    int64_t ldq_f;
    int ncol, nrhs;
    const double *kf;
    int nf;
    int64_t chunk;
    int n_chunks;
    double2 *out;
    int64_t out_fstride;
    int part0;
    int nb;
    bool m3;
};
void launch_mfma64_forward(const Mfma64Job &J, hipStream_t s, PairProfiler *prof);
bool mfma64_nb_ok(int nb);
// 16-target groups per wave: two (one source load and one charge load serve
// 32 targets), except for the double layers with 64 columns per evaluation,
// whose extra source record and FP64 terms leave two groups at one wave per
// SIMD: one group there (measured on c2, 128 columns: 37.2 ms against 42.0 ms
// with two groups, although the loop issues 12% more per pair; the single
// layer took 177.2 ms with one group against 160.5 ms with two)
constexpr int mfma64_groups(int cls, int nb) { return (cls == kClassF && nb == 4) ? 1 : 2; }
void launch_pack_mfma64(SrcClass cls, const SourceSet &src, const double *sp, int64_t sp_fstride, int nf,
                        int nrhs, int ncol, const double2 *x, int64_t ldx, int64_t xfs, double2 *q, int64_t ldq_f,
                        hipStream_t s);
bool mfma_variant_ok(int tg, int nb);
int mfma_grid(int tg, int nb);
// Workgroups (a multiple of 8) that give each wave of an XCD-ranged item list
// at most one item.
int64_t one_item_per_wave_grid(int64_t items);
// q[fl * ldq_f + jj * ncol + col] = scale x[fl * xfs + col * ldx + idx[jj]] for col < nrhs, else 0;
// scale = -s'_f for class G (sp + fl * sp_fstride), 1 for class F
void launch_pack_mfma(SrcClass cls, const SourceSet &src, const double *sp, int64_t sp_fstride, int nf,
                      int nrhs, int ncol, const double2 *x, int64_t ldx, int64_t xfs, float2 *q, int64_t ldq_f,
                      hipStream_t s);

// Single-layer sums among the cells with one evaluation per unordered pair,
// one right-hand side (sym_kernels.hip).  The cells are the canonical points
// 0 .. ng-1 and q their single-layer charges u = -s' x (complex, FP64 or FP32
// per prec).  With vx != null the same evaluations also add the cells'
// adjoint double layer (v' per cell, zero where a cell has none; xv the
// values x; tile_t[t] nonzero when tile t of 64 cells holds a nonzero v').  Cell p receives one partial per group of g 64-point tiles:
// part[slot * ldp + p], slot = 0 .. sym_slots(ng, g) - 1.  Tiles are padded
// with points at far + far_step * lane (farther than the mesh extent from
// every point) and zero charge.
struct SymJob {
    vsie_precision prec;
    int64_t ng;
    const double *px, *py, *pz;
    const void *q;
    double k;
    double far[3];
    double far_step;
    int g;
    void *part;  // slot partials part[slot * ldp + i]: float2 for VSIE_FP32, else double2
    int64_t ldp;
    const double *vx = nullptr, *vy = nullptr, *vz = nullptr;
    const double2 *xv = nullptr;
    const int32_t *tile_t = nullptr;
    const int64_t *xr = nullptr;  // host: 9 item-range boundaries, one range per XCD (null: equal counts)
    // adjoint (needs the T data): q holds conj(lambda) and the partials carry
    // the targets' weights, (-s'_i e + F (x_j - x_i).v'_i) mu_j; sw = s' of the cells
    bool adj = false;
    const double *sw = nullptr;
    int prof_kind = 10;  // profiler kind of the FP64 launch (FP32: + 1)
};
bool sym_groups_ok(int g);
// Item ranges of the 8 XCDs (9 boundaries) with equal modelled work when the
// items whose tiles hold grad-alpha cells (tile_t per 64-cell tile, host)
// cost `weight` times the others: symmetric kernel (ng cells, group size g)
// and cell-face kernel (nc cells, nf faces).
void sym_cost_ranges(int64_t ng, int g, const std::vector<int32_t> &tile_t, double weight, int64_t *xr);
void cf_cost_ranges(int64_t nc, int64_t nf, const std::vector<int32_t> &tile_t, double weight, int64_t *xr);
int64_t sym_slots(int64_t ng, int g);
void launch_sym(const SymJob &J, hipStream_t s, PairProfiler *prof);
// y = diag x + (i < n_vol: sum of the n_slots symmetric partials, float2 when
// sym32, else double2; i >= n_vol: sum of n_face_parts partials over the faces,
// face[c * (n - n_vol) + i - n_vol]) + sum of n_f_parts partials
// fpart[c * n + i]; one right-hand side
void launch_sym_reduce(int64_t n, int64_t n_vol, int n_slots, const void *sym, bool sym32, int64_t ldp,
                       int n_face_parts, const double2 *face, int n_f_parts, const double2 *fpart,
                       const double2 *diag, const double2 *x, double2 *y, hipStream_t s);

// Cell-face pairs with one evaluation per pair, one right-hand side
// (sym_kernels.hip): cells are the points 0 .. nc-1, faces nc .. nc+nf-1; qc
// the cells' single-layer charges, xf the faces' values, vx.. the faces' v'
// (zero where a face has no weight).  With cvx != null the cells' adjoint
// double layer at the faces is added (cvx.. the cells' v', xc their values,
// ctile_t as SymJob::tile_t).  Cell c receives the faces' double layers in
// pc[slot * nc + c] (one slot per group of kCfGroup face tiles), face f the
// cells' single layers in pf[slot * nf + f] (one slot per group of cell tiles).
constexpr int kCfGroup = 2;
struct CfJob {
    vsie_precision prec;
    int64_t nc, nf;
    const double *px, *py, *pz;
    const double *vx, *vy, *vz;
    const void *qc;
    const double2 *xf;
    double k;
    double far[3];
    double far_step;
    void *pc, *pf;  // float2 partials for VSIE_FP32, else double2
    const double *cvx = nullptr, *cvy = nullptr, *cvz = nullptr;
    const double2 *xc = nullptr;
    const int32_t *ctile_t = nullptr;
    const int64_t *xr = nullptr;  // as SymJob::xr
    // adjoint (no grad-alpha cells): qc holds the cells' conj(lambda), qfa the
    // faces' (complex, per prec); cells receive sum e mu_f, faces the face
    // double layer with mu_c
    bool adj = false;
    const void *qfa = nullptr;
    const double *sw = nullptr;  // adjoint with cvx: s' of the cells (weights applied in the kernel)
};
int64_t cf_groups(int64_t count);  // slots for count cells or faces
void launch_cf(const CfJob &J, hipStream_t s, PairProfiler *prof);
// y = diag x + (i < nc: n_sym symmetric slots + n_cs cell slots of pc;
// i >= nc: n_fs face slots of pf + n_ff face-face chunk partials ff[c * nf + i - nc]);
// sym, pc and pf hold float2 partials when slots32, else double2; ff holds
// float2 when ff32, else double2;
// adj: y = conj(diag) x + conj(w sum) with w = -s'_i for cells when adj_sp
// (the frequency's s' of all points) is given, else 1
void launch_cf_reduce(int64_t n, int64_t nc, bool slots32, int n_sym, const void *sym, int n_cs, const void *pc,
                      int n_fs, const void *pf, int n_ff, const void *ff, bool ff32, const double2 *diag,
                      const double2 *x, double2 *y, hipStream_t s, bool adj = false, const double *adj_sp = nullptr);

// Product with the assembled FP32 operator on the matrix cores
// (dense_kernels.hip), nrhs <= kDenseCols columns:
//   forward y = d x + A x,  adjoint y = conj(d) x + A^H x,
// A in two column-major FP32 planes ar, ai (leading dimension ld).  FP32 sums
// over slabs of kDenseSlab sources, added in FP64 in slab order.  Work
// buffers: xp (2 dense_npad(n) kDenseCols floats, the packed columns) and part
// (ceil(n / kDenseSlab) nrhs n double2, the slab partials).
constexpr int kDenseCols = 128;
constexpr int64_t kDenseSlab = 8192;
struct DenseJob {
    bool adjoint, m3;
    int64_t n;
    const float *ar, *ai;
    int64_t ld;
    int nrhs;
    const double2 *x;
    int64_t ldx;
    float *xp;
    double2 *part;
    const double2 *diag;
    double2 *y;
    int64_t ldy;
};
int64_t dense_npad(int64_t n);
void launch_dense_product(const DenseJob &J, hipStream_t s, PairProfiler *prof);

// auxiliary kernels (aux_kernels.hip)
void launch_weights(const DeviceMesh &m, const double *k0, int n_freq, hipStream_t s);
// charge[r * count + jj] = scale * x[idx[jj] + r ldx], scale = -s'_f for class G, else 1
void launch_pack_charges(SrcClass cls, vsie_precision prec, const SourceSet &src,
                         const double *sp_f, int nrhs, const double2 *x, int64_t ldx,
                         bool conj_in, void *charge, hipStream_t s);
// launch_pack_charges for both classes (G with sp_f) in one launch
void launch_pack_both(vsie_precision prec, const SourceSet &G, const SourceSet &F, const double *sp_f, int nrhs,
                      const double2 *x, int64_t ldx, bool conj_in, void *chargeG, void *chargeF, hipStream_t s);
// charge[r * n + j] = x[j + r ldx] (conjugated when conj_in)
void launch_pack_plain(vsie_precision prec, int64_t n, int nrhs, const double2 *x, int64_t ldx,
                       bool conj_in, void *charge, hipStream_t s);
// y = diag * x + sum of n_parts partial blocks (diag may be null)
void launch_reduce_partials(int64_t n_t, int nrhs, int n_parts, const double2 *partial,
                            const double2 *diag, bool conj_diag, const double2 *x, int64_t ldx,
                            double2 *y, int64_t ldy, double2 *unused, hipStream_t s);
// X2 (n x 2 nrhs FP32, column-major, leading dimension n) = [Re x | Im x]
void launch_pack_planar(int64_t n, int nrhs, const double2 *x, int64_t ldx, float *X2, hipStream_t s);
// y = d x + the FP64 sum over n_parts slabs of the planar FP32 partial products:
// slab c holds P = Ar_c X2 and then Q = Ai_c X2 (n x 2 nrhs each, leading
// dimension n; transposed slabs of A for the adjoint), combined as
// forward  y = d x + sum_c (P_r - Q_i) + i (P_i + Q_r),
// adjoint  y = conj(d) x + sum_c (P_r + Q_i) + i (P_i - Q_r),
// where _r and _i are the column blocks of X2's real and imaginary parts.
void launch_reduce_planar(int64_t n, int nrhs, int n_parts, const float *partial, const double2 *diag,
                          bool adjoint, const double2 *x, int64_t ldx, double2 *y, int64_t ldy, hipStream_t s);
// dense FP32 off-diagonal operator in two planes, real parts A[i + j ld] and
// imaginary parts A[ld n + i + j ld], column-major (pair_kernels.hip)
void launch_assemble_dense(int64_t n, const double *px, const double *py, const double *pz,
                           const double *sp, const double *vpx, const double *vpy, const double *vpz,
                           double k, float *A, int64_t ld, hipStream_t s);
// y[idx[jj]] += conj(scale * sum of partials), scale = -s' (sp != null) or 1
void launch_scatter_conj(int64_t count, const int32_t *idx, const double *sp, int nrhs,
                         int n_parts, const double2 *partial, double2 *y, int64_t ldy,
                         hipStream_t s);
void launch_sums_reduce(int64_t n, int nrhs, int n_parts, const double2 *partial, double2 *z,
                        int64_t ldz, double2 *Z, int64_t ldZ, hipStream_t s);
void launch_plane_wave(int64_t n, const double *px, const double *py, const double *pz, double k,
                       double dx, double dy, double dz, double2 *b, hipStream_t s);

// adjoint-state gradient (gradient.hip)
void launch_adjoint_rhs(const DeviceMesh &m, int f, int nrhs, const double2 *zR, int64_t ldz,
                        const double2 *ZR, int64_t ldZ, double2 *out, int64_t ldo, hipStream_t s);
void launch_param_gradient(const DeviceMesh &m, const int32_t *cf_off, const int32_t *cf_idx,
                           double k, int nrhs, const double2 *P, int64_t ldp, const double2 *L,
                           int64_t ldl, const double2 *z, int64_t ldz, const double2 *Z, int64_t ldZ,
                           const double2 *zR, int64_t ldzr, const double2 *ZR, int64_t ldZr,
                           double *work, double *grad_c, double *grad_rho, hipStream_t s);
void launch_plane_wave_at(int64_t n, const double *tx, const double *ty, const double *tz, double k,
                          double dx, double dy, double dz, double2 *b, hipStream_t s);

// dense vector kernels for the Krylov solver (aux_kernels.hip)
void blas_zero(int64_t n, double2 *v, hipStream_t s);

// batched Krylov kernels (aux_kernels.hip); basis vector j of rhs r at V + (j R + r) n
void bblas_dots(int64_t n, int k, int R, int nslots, const int32_t *act, const double2 *V,
                const double2 *W, double2 *partial, int n_chunks, double2 *h, int hstride,
                hipStream_t s);
void bblas_gemv_sub(int64_t n, int k, int R, int nslots, const int32_t *act, const double2 *V,
                    const double2 *h, int hstride, double2 *W, hipStream_t s,
                    const int32_t *kd = nullptr);
void bblas_norm(int64_t n, int nslots, const double2 *W, double *partial, int n_chunks, double *out,
                hipStream_t s);
void bblas_scale_into_basis(int64_t n, int kcol, int R, int nslots, const int32_t *act,
                            const double2 *W, const double *nrm, double2 *V, hipStream_t s);
// The same Arnoldi step in fewer launches: projections to chunk partials, then
// the update that sums them itself (and stores the coefficients in h); norm
// partials, then the scaling that sums them itself (and stores the norms).
// The update needs k <= 1024 (bblas_fused_ok).
bool bblas_fused_ok(int k);
void bblas_dots_partial(int64_t n, int k, int R, int nslots, const int32_t *act, const double2 *V,
                        const double2 *W, double2 *partial, int n_chunks, hipStream_t s);
void bblas_gemv_sub_partial(int64_t n, int k, int R, int nslots, const int32_t *act, const double2 *V,
                            const double2 *partial, int n_chunks, double2 *h, int hstride, double2 *W,
                            hipStream_t s);
void bblas_norm_partial(int64_t n, int nslots, const double2 *W, double *partial, int n_chunks, hipStream_t s);
void bblas_norm_scale(int64_t n, int kcol, int R, int nslots, const int32_t *act, const double2 *W,
                      const double *partial, int n_chunks, double *nrm, double2 *V, hipStream_t s);
void bblas_gather(int64_t n, int nslots, const int32_t *act, const double2 *src, int64_t ld,
                  double2 *X, hipStream_t s);
// Deflation coefficients of one Gram-Schmidt pass for nl live right-hand
// sides: live position l holds slot sl = slot[l] with kc = kcount[sl] recycled
// vectors (0: none) and projections t = tc[l * cs + 0..kc).  With P and M the
// slot's kc x kc and (kc - 1) x kc matrices (column-major, leading dimension
// cs, at P + sl * cs * cs and M + sl * cs * cs):
//   hc[l * cs + i] = (P t)_i                       i < kc (0 up to cs)
//   B[sl * bstride + col * kb + i] += (M t)_i      i < kc - 1
void bblas_deflate_coef(int nl, const int32_t *slot, const int32_t *kcount, int cs, const double2 *P,
                        const double2 *M, const double2 *tc, double2 *hc, double2 *B, int col, int kb,
                        int64_t bstride, hipStream_t s);
void bblas_update(int64_t n, int R, int nslots, const int32_t *act, const int32_t *kd, const double2 *V,
                  const double2 *y, int ystride, double2 *x, int64_t ldx, hipStream_t s);
void blas_scatter_add(int64_t n, int nslots, const int32_t *act, const double2 *W, double2 *x, int64_t ldx,
                      hipStream_t s);
// C (m x nn, leading dimension ldc) = sum of parts consecutive m x nn column-major slabs of P
void blas_sum_slabs(int64_t m, int64_t nn, int parts, const double2 *P, double2 *C, int64_t ldc, hipStream_t s);
// Tall-skinny block products for blocks of at most kTsMaxCols columns (see
// ts_cn_kernel and ts_nn_kernel): C (m x nn) = A^H B with A rows x m and B
// rows x nn, through ts_cn_bytes(m, nn, rows) bytes of slab partials P; and
// C = alpha A B (+ C when accumulate) with A rows x k, B k x nn on the device.
constexpr int kTsMaxCols = 32;
size_t ts_cn_bytes(int64_t m, int64_t nn, int64_t rows);
void ts_cn(int64_t rows, int64_t m, int64_t nn, const double2 *A, int64_t lda, const double2 *B, int64_t ldb,
           double2 *P, double2 *C, int64_t ldc, hipStream_t s);
void ts_nn(int64_t rows, int64_t k, int64_t nn, double alpha, bool accumulate, const double2 *A, int64_t lda,
           const double2 *B, int64_t ldb, double2 *C, int64_t ldc, hipStream_t s);
// Cholesky factor G = T^H T of a Hermitian r x r Gram matrix on the device
// (r <= kSmallChol, one workgroup), with T^{-1} and optionally T Tprev; see
// small_chol_kernel for the shift and the status codes.
constexpr int kSmallChol = 32;
void launch_small_chol(const double2 *G, int r, double2 *T, double2 *Ti, const double2 *Tprev, double2 *Tout,
                       int *status, hipStream_t s);
void bblas_sub(int64_t n, int nslots, const int32_t *act, const double2 *b, int64_t ldb,
               const double2 *ax, double2 *out, hipStream_t s);

}  // namespace vsie
