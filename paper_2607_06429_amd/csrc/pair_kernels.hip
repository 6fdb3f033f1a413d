// Pair-sum kernels of the discretised VSIE operator on gfx950.
//
// One thread owns one "thread point" (a collocation target in the forward
// product, a source element in the adjoint sums) and streams a chunk of
// "streamed points".  The streamed index is the same for every lane of a
// wave, so their coordinates, weights and charges are read with wave-uniform
// (scalar) loads straight from global memory: no LDS staging and no
// barriers.  Chunks of streamed points are spread over blockIdx.y so that a
// launch holds many more waves than the chip has SIMDs; each (thread point,
// chunk) writes one FP64 partial sum per right-hand side and a separate
// kernel adds the partials in a fixed order (deterministic results).
//
// Per pair, with d = x_thread - y_streamed, r = |d| (paper: the midpoint rule
// applied to the kernels of Theorem 3, eq_vsie, with G = exp(i k r)/(4 pi r)):
//   e      = exp(i k r) / r                  (the 1/(4 pi) lives in the weights)
//   FWD_G  : acc += e * u_j                  single layer, u_j = -s'_j x_j
//   FWD_F  : acc += e (i k r - 1) q * x_j,   q = d . v'_j / r^2   (T and K terms)
//   ADJ_F  : acc += e (i k r - 1) q * c_j,   q = -d . v'_thread / r^2
//   SUMS   : z   += e * c_j,  Zvec += e (i k r - 1)/r^2 (-d) * c_j
// A pair with r = 0 (the thread point itself) contributes exactly zero.
//
// Phase: the angle k r is carried in revolutions t = r k/(2 pi), reduced as
// t - rint(t) in FP64 on both precision paths, so the argument of sin/cos
// never exceeds half a turn.
#include <type_traits>

#include "pair_geom.h"
#include "vsie_internal.h"

namespace vsie {
namespace {

using namespace geom;

enum Mode { FWD_G = 0, FWD_F = 1, ADJ_F = 2, SUMS = 3 };

template <typename CT, typename AT>
struct PairArgs {
    int64_t n_t;
    const CT *__restrict__ tx;
    const CT *__restrict__ ty;
    const CT *__restrict__ tz;
    const double *__restrict__ tvx;  // ADJ_F: v' of the thread points
    const double *__restrict__ tvy;
    const double *__restrict__ tvz;
    int64_t n_s;
    const CT *__restrict__ sx;
    const CT *__restrict__ sy;
    const CT *__restrict__ sz;
    const double *__restrict__ svx;  // FWD_F: v' of the streamed points
    const double *__restrict__ svy;
    const double *__restrict__ svz;
    const void *__restrict__ q;  // charges, complex pairs of AT: q[r * ldq + j]
    int64_t ldq;
    int64_t chunk;
    double k;
    double kphase;               // k/pi (FP64: half turns) or k/(2 pi) (FP32: turns)
    double2 *__restrict__ out;   // out[c * chunk_stride + (r * ncomp + comp) * n_t + i]
    int64_t chunk_stride;
    int self_mode;               // which streamed points may coincide with a thread point
    const int32_t *__restrict__ self_idx;  // canonical indices of the class entries
};

template <typename AT> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };

// Sources per FP32 sub-tile: FP32 sums over at most this many pairs are
// added into the FP64 accumulators.
constexpr int kSubTile = 128;

// first position in the increasing array a[0..n) holding a value >= v
__device__ int64_t lower_bound_u(const int32_t *__restrict__ a, int64_t n, int64_t v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Streamed points per unrolled step of the pair loop: four while their
// wave-uniform charges are small (fewer scalar address updates and waits per
// pair), else two (the charges of more steps would not fit the scalar
// registers).
template <int R, typename AT>
constexpr int pair_unroll() {
    return R * static_cast<int>(sizeof(AT) / 4) < 4 ? 4 : 2;
}

template <int MODE, int R, typename CT, typename AT>
__global__ __launch_bounds__(kBlock) void pair_sum_kernel(PairArgs<CT, AT> a) {
    using C2 = typename cplx_t<AT>::type;
    constexpr int NC = (MODE == SUMS) ? 4 : 1;   // complex accumulators per right-hand side
    constexpr bool F32 = sizeof(AT) == 4;
    const int64_t wave0 = static_cast<int64_t>(blockIdx.x) * kBlock +
                          64 * __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (wave0 >= a.n_t) return;  // whole wave outside (a partial wave clamps below)
    const bool active = i < a.n_t;
    const int64_t ii = active ? i : a.n_t - 1;
    const int c = blockIdx.y;
    const int64_t j0 = static_cast<int64_t>(c) * a.chunk;
    const int64_t j1 = (j0 + a.chunk < a.n_s) ? j0 + a.chunk : a.n_s;

    // Streamed indices [sr0, sr1) that may coincide with one of this wave's
    // thread points; only there is the pair r = 0 masked.
    const int64_t wlast = (wave0 + 63 < a.n_t) ? wave0 + 63 : a.n_t - 1;
    int64_t sr0 = 0, sr1 = 0;
    switch (a.self_mode) {
        case SELF_NONE: sr0 = 0; sr1 = a.n_s; break;   // unknown targets: mask everything
        case SELF_IDENT: sr0 = wave0; sr1 = wlast + 1; break;
        case SELF_STREAM_IDX:
            sr0 = lower_bound_u(a.self_idx, a.n_s, wave0);
            sr1 = lower_bound_u(a.self_idx, a.n_s, wlast + 1);
            break;
        case SELF_THREAD_IDX: sr0 = a.self_idx[wave0]; sr1 = a.self_idx[wlast] + 1; break;
        default: break;
    }
    const int64_t m0 = sr0 > j0 ? sr0 : j0;
    const int64_t m1 = sr1 < j1 ? sr1 : j1;

    const double xi = a.tx[ii], yi = a.ty[ii], zi = a.tz[ii];
    double tv0 = 0, tv1 = 0, tv2 = 0;
    if constexpr (MODE == ADJ_F) {
        tv0 = a.tvx[ii];
        tv1 = a.tvy[ii];
        tv2 = a.tvz[ii];
    }
    const C2 *__restrict__ q = static_cast<const C2 *>(a.q);

    double accr[R * NC], acci[R * NC];
#pragma unroll
    for (int r = 0; r < R * NC; ++r) accr[r] = acci[r] = 0.0;

    const AT k = static_cast<AT>(a.k);
    // Sum over streamed points [ja, jb), in FP32 sub-tiles on the FP32 path.
    auto run = [&](int64_t ja, int64_t jb, auto mask_tag) {
        constexpr bool MASK = decltype(mask_tag)::value;
        for (int64_t jt = ja; jt < jb; jt += (F32 ? kSubTile : (jb - ja))) {
            const int64_t je = F32 ? ((jt + kSubTile < jb) ? jt + kSubTile : jb) : jb;
            AT sr[R * NC], si[R * NC];
#pragma unroll
            for (int r = 0; r < R * NC; ++r) sr[r] = si[r] = 0;
#pragma unroll pair_unroll<R, AT>()
            for (int64_t j = jt; j < je; ++j) {
                const double dx = xi - static_cast<double>(a.sx[j]);
                const double dy = yi - static_cast<double>(a.sy[j]);
                const double dz = zi - static_cast<double>(a.sz[j]);
                AT er, ei, ir2, kr;
                if constexpr (F32) geom_f32<MASK>(dx, dy, dz, k, a.kphase, er, ei, ir2, kr);
                else geom_f64<MASK>(dx, dy, dz, a.k, a.kphase, er, ei, ir2, kr);
                if constexpr (MODE == FWD_G) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const C2 u = q[r * a.ldq + j];
                        sr[r] = fma(er, u.x, fma(-ei, u.y, sr[r]));
                        si[r] = fma(er, u.y, fma(ei, u.x, si[r]));
                    }
                } else if constexpr (MODE == FWD_F || MODE == ADJ_F) {
                    AT dv;
                    // (x_thread - y_streamed) . v' in FP64 (v' kept in FP64 on both paths)
                    if constexpr (MODE == FWD_F) {
                        dv = static_cast<AT>(fma(dx, a.svx[j], fma(dy, a.svy[j], dz * a.svz[j])));
                    } else {
                        dv = -static_cast<AT>(fma(dx, tv0, fma(dy, tv1, dz * tv2)));
                    }
                    const AT qq = dv * ir2;
                    // e (i k r - 1) q
                    const AT cr = qq * fma(-ei, kr, -er);
                    const AT ci = qq * fma(er, kr, -ei);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const C2 u = q[r * a.ldq + j];
                        sr[r] = fma(cr, u.x, fma(-ci, u.y, sr[r]));
                        si[r] = fma(cr, u.y, fma(ci, u.x, si[r]));
                    }
                } else {  // SUMS
                    const AT cr = ir2 * fma(-ei, kr, -er);
                    const AT ci = ir2 * fma(er, kr, -ei);
                    const AT md[3] = {static_cast<AT>(-dx), static_cast<AT>(-dy), static_cast<AT>(-dz)};
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const C2 u = q[r * a.ldq + j];
                        sr[4 * r] = fma(er, u.x, fma(-ei, u.y, sr[4 * r]));
                        si[4 * r] = fma(er, u.y, fma(ei, u.x, si[4 * r]));
                        const AT wr = fma(cr, u.x, -ci * u.y);
                        const AT wi = fma(cr, u.y, ci * u.x);
#pragma unroll
                        for (int ax = 0; ax < 3; ++ax) {
                            sr[4 * r + 1 + ax] = fma(md[ax], wr, sr[4 * r + 1 + ax]);
                            si[4 * r + 1 + ax] = fma(md[ax], wi, si[4 * r + 1 + ax]);
                        }
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R * NC; ++r) {
                accr[r] += static_cast<double>(sr[r]);
                acci[r] += static_cast<double>(si[r]);
            }
        }
    };
    if (m0 >= m1) {
        run(j0, j1, std::false_type{});
    } else {
        run(j0, m0, std::false_type{});
        run(m0, m1, std::true_type{});
        run(m1, j1, std::false_type{});
    }
    if (!active) return;
    double2 *__restrict__ o = a.out + c * a.chunk_stride + i;
#pragma unroll
    for (int r = 0; r < R * NC; ++r) o[r * a.n_t] = make_double2(accr[r], acci[r]);
}

template <int MODE, typename CT, typename AT>
void launch_mode(const PairArgs<CT, AT> &a, int nrhs, int n_chunks, hipStream_t s) {
    dim3 grid(static_cast<unsigned>((a.n_t + kBlock - 1) / kBlock), static_cast<unsigned>(n_chunks));
    switch (nrhs) {
        case 1: hipLaunchKernelGGL((pair_sum_kernel<MODE, 1, CT, AT>), grid, dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((pair_sum_kernel<MODE, 2, CT, AT>), grid, dim3(kBlock), 0, s, a); break;
        case 4: hipLaunchKernelGGL((pair_sum_kernel<MODE, 4, CT, AT>), grid, dim3(kBlock), 0, s, a); break;
        case 8: hipLaunchKernelGGL((pair_sum_kernel<MODE, 8, CT, AT>), grid, dim3(kBlock), 0, s, a); break;
        case 16: hipLaunchKernelGGL((pair_sum_kernel<MODE, 16, CT, AT>), grid, dim3(kBlock), 0, s, a); break;
        default: fail(VSIE_E_INVALID, "pair kernel: unsupported right-hand-side block " + std::to_string(nrhs));
    }
    VSIE_HIP(hipGetLastError());
}

// Dense FP32 off-diagonal operator: A[i + j ld] = kappa(x_i, y_j) for the
// sources j in [j0, j0 + jcount) of this launch, kappa = e (-s'_j + q_ij (i k r - 1)),
// e = exp(i k r)/r, q_ij = (x_i - y_j).v'_j / r^2, computed with the FP64 pair
// geometry and rounded once to FP32; the diagonal entries are 0.
__global__ __launch_bounds__(kBlock) void assemble_kernel(
    int64_t n, const double *__restrict__ px, const double *__restrict__ py,
    const double *__restrict__ pz, const double *__restrict__ sp, const double *__restrict__ vpx,
    const double *__restrict__ vpy, const double *__restrict__ vpz, double k, double khalf,
    float *__restrict__ Ar, float *__restrict__ Ai, int64_t ld, int64_t chunk) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t j0 = static_cast<int64_t>(blockIdx.y) * chunk;
    const int64_t j1 = (j0 + chunk < n) ? j0 + chunk : n;
    const double xi = px[i], yi = py[i], zi = pz[i];
    for (int64_t j = j0; j < j1; ++j) {
        const double dx = xi - px[j], dy = yi - py[j], dz = zi - pz[j];
        double er, ei, ir2, kr;
        geom_f64<true>(dx, dy, dz, k, khalf, er, ei, ir2, kr);
        const double q = fma(dx, vpx[j], fma(dy, vpy[j], dz * vpz[j])) * ir2;
        // e * (-s' - q + i k r q)
        const double br = -sp[j] - q, bi = kr * q;
        Ar[i + j * ld] = static_cast<float>(er * br - ei * bi);
        Ai[i + j * ld] = static_cast<float>(er * bi + ei * br);
    }
}

}  // namespace

void launch_assemble_dense(int64_t n, const double *px, const double *py, const double *pz,
                           const double *sp, const double *vpx, const double *vpy, const double *vpz,
                           double k, float *A, int64_t ld, hipStream_t s) {
    if (n == 0) return;
    const int64_t chunk = 512;
    dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock), static_cast<unsigned>((n + chunk - 1) / chunk));
    hipLaunchKernelGGL(assemble_kernel, grid, dim3(kBlock), 0, s, n, px, py, pz, sp, vpx, vpy, vpz, k,
                       k / kPi, A, A + ld * n, ld, chunk);
    VSIE_HIP(hipGetLastError());
}

// Splits nrhs into launches of 16, 8, 4, 2, 1 right-hand sides.
template <int MODE>
static void run_pairs(const PairJob &J, hipStream_t s) {
    constexpr int NC = (MODE == SUMS) ? 4 : 1;
    const double kphase = (J.prec == VSIE_FP64) ? J.k / kPi : J.k / kTwoPi;
    int r0 = 0;
    while (r0 < J.nrhs) {
        const int left = J.nrhs - r0;
        const int blk = left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
        double2 *out = J.out + static_cast<int64_t>(r0) * NC * J.n_t;
        if (J.prec == VSIE_FP64) {
            PairArgs<double, double> a{J.n_t, J.tx, J.ty, J.tz, J.tv[0], J.tv[1], J.tv[2],
                                       J.n_s, J.sx, J.sy, J.sz, J.sv[0], J.sv[1], J.sv[2],
                                       static_cast<const double2 *>(J.charge) + r0 * J.ldq, J.ldq,
                                       J.chunk, J.k, kphase, out, J.chunk_stride, J.self_mode,
                                       J.self_idx};
            launch_mode<MODE>(a, blk, J.n_chunks, s);
        } else {
            PairArgs<double, float> a{J.n_t, J.tx, J.ty, J.tz, J.tv[0], J.tv[1], J.tv[2],
                                      J.n_s, J.sx, J.sy, J.sz, J.sv[0], J.sv[1], J.sv[2],
                                      static_cast<const float2 *>(J.charge) + r0 * J.ldq, J.ldq,
                                      J.chunk, J.k, kphase, out, J.chunk_stride, J.self_mode,
                                      J.self_idx};
            launch_mode<MODE>(a, blk, J.n_chunks, s);
        }
        r0 += blk;
    }
}

hipEvent_t prof_take_event(PairProfiler *prof) {
    if (!prof->pool.empty()) {
        hipEvent_t e = prof->pool.back();
        prof->pool.pop_back();
        return e;
    }
    hipEvent_t e;
    VSIE_HIP(hipEventCreate(&e));
    return e;
}

void launch_pairs(const PairJob &J, hipStream_t s, PairProfiler *prof) {
    if (J.n_t == 0 || J.n_s == 0) return;
    if (J.chunk <= 0 || J.n_chunks <= 0 || (J.n_chunks - 1) * J.chunk >= J.n_s)
        fail(VSIE_E_INVALID, "pair kernel: inconsistent source chunking");
    if (prof && prof->on) {
        PairProfiler::Rec r{prof_take_event(prof), prof_take_event(prof), 2 * J.mode + (J.prec == VSIE_FP32 ? 1 : 0),
                            static_cast<double>(J.n_t) * J.n_s,
                            static_cast<double>(J.n_t) * J.n_s * J.nrhs};
        VSIE_HIP(hipEventRecord(r.a, s));
        PairJob K = J;
        launch_pairs(K, s, nullptr);
        VSIE_HIP(hipEventRecord(r.b, s));
        prof->recs.push_back(r);
        return;
    }
    switch (J.mode) {
        case PAIR_FWD_G: run_pairs<FWD_G>(J, s); break;
        case PAIR_FWD_F: run_pairs<FWD_F>(J, s); break;
        case PAIR_ADJ_F: run_pairs<ADJ_F>(J, s); break;
        case PAIR_SUMS: run_pairs<SUMS>(J, s); break;
        default: fail(VSIE_E_INVALID, "pair kernel: unknown mode");
    }
}

}  // namespace vsie
