// Far-field pattern of the scattered pressure on gfx950.
//
// The exterior field of section 2.3.1 is p(x) = p_inc(x) - sum_j A(x, j) x_j.
// Along a unit direction d, with x = R d and R -> infinity, the kernels reduce
// to their leading terms
//   exp(i k r)/r           -> exp(i k R)/R exp(-i k d.y)
//   exp(i k r)(i k r - 1) (x - y).v'/r^3 -> exp(i k R)/R exp(-i k d.y) i k d.v'
// so p - p_inc = exp(i k R)/R pinf(d) + O(R^-2) with
//   pinf(d) = -sum_G exp(-i k d.y_j) u_j - sum_F exp(-i k d.y_j) i k (d.v'_j) x_j,
// where u_j = -s'_j x_j are the single-layer charges of the forward product
// (class G) and the class F entries carry v' (the T and K weights), both
// already divided by 4 pi.
//
// A lane owns one or two directions and streams a chunk of sources; the
// source index is the same for every lane of a wave, so the packed source
// records (x, y, z, 0), (v', 0) and the charges come from wave-uniform loads,
// each serving every direction of the lane.  Chunks of sources are spread over blockIdx.y
// and each (chunk, right-hand side, direction) writes one FP64 partial; the
// caller adds the partials in a fixed order.  The phase -k d.y is formed in
// FP64 on both precision paths and reduced exactly before sin and cos: to
// turns with v_fract_f64 and the FP32 v_sin/v_cos (which take turns) on the
// FP32 path, to half turns around rint with the FP64 series of the pair
// geometry on the FP64 path.  FP32 sums run over at most 128 sources before
// they are added in FP64.
#include "pair_geom.h"
#include "vsie_internal.h"

namespace vsie {
namespace {

using namespace geom;

template <typename AT>
struct FarArgs {
    int64_t n_d;
    const double *__restrict__ dx;
    const double *__restrict__ dy;
    const double *__restrict__ dz;
    int64_t n_s;
    const double4 *__restrict__ pk;  // (x, y, z, 0) of the sources
    const double4 *__restrict__ pv;  // class F: (v'x, v'y, v'z, 0)
    const void *__restrict__ q;      // complex charges of AT: q[r * ldq + j]
    int64_t ldq;
    int64_t chunk;
    double k;
    double kphase;                   // k/pi (FP64: half turns) or k/(2 pi) (FP32: turns)
    double2 *__restrict__ out;       // out[c * chunk_stride + r * n_d + i]
    int64_t chunk_stride;
};

template <typename AT> struct far_cplx;
template <> struct far_cplx<double> { using type = double2; };
template <> struct far_cplx<float> { using type = float2; };

constexpr int kFarSubTile = 128;

// Directions per lane: two for up to four right-hand sides (each source's
// wave-uniform loads then serve two pairs per lane), one above.
constexpr int far_lanes(int R) { return R <= 4 ? 2 : 1; }

// Lane l of workgroup b owns directions b * kBlock * TPL + u * kBlock + l,
// u < TPL (each u coalesced across the wave).
template <int CLS, int R, typename AT>
__global__ __launch_bounds__(kBlock) void far_field_kernel(FarArgs<AT> a) {
    using C2 = typename far_cplx<AT>::type;
    constexpr bool F32 = sizeof(AT) == 4;
    constexpr int TPL = far_lanes(R);
    // sources per unrolled step: their wave-uniform charges (R complex each)
    // must fit the scalar registers
    constexpr int LOAD = R * (CLS == kClassF ? 2 : 1);
    constexpr int UNR = LOAD >= 16 ? 1 : LOAD >= 4 ? 2 : 4;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kBlock * TPL;
    const int64_t wave0 = base + 64 * __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    if (wave0 >= a.n_d) return;  // every direction of the wave is outside (a partial wave clamps below)
    const int c = blockIdx.y;
    const int64_t j0 = static_cast<int64_t>(c) * a.chunk;
    const int64_t j1 = (j0 + a.chunk < a.n_s) ? j0 + a.chunk : a.n_s;
    // per direction: -kphase d (the phase in turns or half turns is w . y) and k d
    double wx[TPL], wy[TPL], wz[TPL], kx[TPL], ky[TPL], kz[TPL];
#pragma unroll
    for (int u = 0; u < TPL; ++u) {
        const int64_t t = base + u * kBlock + threadIdx.x;
        const int64_t tt = t < a.n_d ? t : a.n_d - 1;
        const double ux = a.dx[tt], uy = a.dy[tt], uz = a.dz[tt];
        wx[u] = -a.kphase * ux;
        wy[u] = -a.kphase * uy;
        wz[u] = -a.kphase * uz;
        kx[u] = a.k * ux;
        ky[u] = a.k * uy;
        kz[u] = a.k * uz;
    }
    const C2 *__restrict__ q = static_cast<const C2 *>(a.q);

    double accr[TPL][R], acci[TPL][R];
#pragma unroll
    for (int u = 0; u < TPL; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) accr[u][r] = acci[u][r] = 0.0;

    for (int64_t jt = j0; jt < j1; jt += (F32 ? kFarSubTile : (j1 - j0))) {
        const int64_t je = F32 ? ((jt + kFarSubTile < j1) ? jt + kFarSubTile : j1) : j1;
        AT sr[TPL][R], si[TPL][R];
#pragma unroll
        for (int u = 0; u < TPL; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r) sr[u][r] = si[u][r] = 0;
#pragma unroll UNR
        for (int64_t j = jt; j < je; ++j) {
            const double4 y = a.pk[j];
            double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
            if constexpr (CLS == kClassF) v = a.pv[j];
            C2 qv[R];
#pragma unroll
            for (int r = 0; r < R; ++r) qv[r] = q[r * a.ldq + j];
#pragma unroll
            for (int u = 0; u < TPL; ++u) {
                // exp(-i k d.y) = (er, ei) from the FP64 phase w . y
                const double ph = fma(wx[u], y.x, fma(wy[u], y.y, wz[u] * y.z));
                AT er, ei;
                if constexpr (F32) {
                    const float f = static_cast<float>(__builtin_amdgcn_fract(ph));
                    er = __builtin_amdgcn_cosf(f);
                    ei = __builtin_amdgcn_sinf(f);
                } else {
                    const double qn = rint(ph);
                    double sn, cs;
                    sincos_halfturn_f64(ph - qn, sn, cs);
                    er = flip_if_odd(cs, qn);
                    ei = flip_if_odd(sn, qn);
                }
                AT wr, wi;
                if constexpr (CLS == kClassG) {
                    wr = er;
                    wi = ei;
                } else {
                    // exp(-i k d.y) * i k (d . v')
                    const AT kd = static_cast<AT>(fma(kx[u], v.x, fma(ky[u], v.y, kz[u] * v.z)));
                    wr = -ei * kd;
                    wi = er * kd;
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    sr[u][r] = fma(wr, qv[r].x, fma(-wi, qv[r].y, sr[u][r]));
                    si[u][r] = fma(wr, qv[r].y, fma(wi, qv[r].x, si[u][r]));
                }
            }
        }
#pragma unroll
        for (int u = 0; u < TPL; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                accr[u][r] += static_cast<double>(sr[u][r]);
                acci[u][r] += static_cast<double>(si[u][r]);
            }
    }
#pragma unroll
    for (int u = 0; u < TPL; ++u) {
        const int64_t t = base + u * kBlock + threadIdx.x;
        if (t >= a.n_d) continue;
        double2 *__restrict__ o = a.out + c * a.chunk_stride + t;
#pragma unroll
        for (int r = 0; r < R; ++r) o[r * a.n_d] = make_double2(-accr[u][r], -acci[u][r]);
    }
}

template <int CLS, int R, typename AT>
void launch_one(const FarArgs<AT> &a, int n_chunks, hipStream_t s) {
    const int64_t per_block = static_cast<int64_t>(kBlock) * far_lanes(R);
    dim3 grid(static_cast<unsigned>((a.n_d + per_block - 1) / per_block), static_cast<unsigned>(n_chunks));
    hipLaunchKernelGGL((far_field_kernel<CLS, R, AT>), grid, dim3(kBlock), 0, s, a);
}

template <int CLS, typename AT>
void launch_block(const FarArgs<AT> &a, int nrhs, int n_chunks, hipStream_t s) {
    switch (nrhs) {
        case 1: launch_one<CLS, 1>(a, n_chunks, s); break;
        case 2: launch_one<CLS, 2>(a, n_chunks, s); break;
        case 4: launch_one<CLS, 4>(a, n_chunks, s); break;
        case 8: launch_one<CLS, 8>(a, n_chunks, s); break;
        case 16: launch_one<CLS, 16>(a, n_chunks, s); break;
        default: fail(VSIE_E_INVALID, "far-field kernel: unsupported right-hand-side block " + std::to_string(nrhs));
    }
    VSIE_HIP(hipGetLastError());
}

// Splits nrhs into launches of 16, 8, 4, 2, 1 right-hand sides.
template <int CLS>
void run_far(const FarJob &J, hipStream_t s) {
    const double kphase = (J.prec == VSIE_FP64) ? J.k / kPi : J.k / kTwoPi;
    int r0 = 0;
    while (r0 < J.nrhs) {
        const int left = J.nrhs - r0;
        const int blk = left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
        double2 *out = J.out + static_cast<int64_t>(r0) * J.n_d;
        if (J.prec == VSIE_FP64) {
            FarArgs<double> a{J.n_d, J.dx, J.dy, J.dz, J.n_s, J.pk, J.pv,
                              static_cast<const double2 *>(J.charge) + r0 * J.ldq, J.ldq, J.chunk, J.k, kphase,
                              out, J.chunk_stride};
            launch_block<CLS>(a, blk, J.n_chunks, s);
        } else {
            FarArgs<float> a{J.n_d, J.dx, J.dy, J.dz, J.n_s, J.pk, J.pv,
                             static_cast<const float2 *>(J.charge) + r0 * J.ldq, J.ldq, J.chunk, J.k, kphase,
                             out, J.chunk_stride};
            launch_block<CLS>(a, blk, J.n_chunks, s);
        }
        r0 += blk;
    }
}

}  // namespace

int far_field_lanes(int nrhs) { return far_lanes(nrhs >= 16 ? 16 : nrhs >= 8 ? 8 : nrhs); }

void launch_far_field(const FarJob &J, hipStream_t s, PairProfiler *prof) {
    if (J.n_d == 0 || J.n_s == 0) return;
    if (J.chunk <= 0 || J.n_chunks <= 0 || (J.n_chunks - 1) * J.chunk >= J.n_s)
        fail(VSIE_E_INVALID, "far-field kernel: inconsistent source chunking");
    if (!J.pk || (J.cls == kClassF && !J.pv)) fail(VSIE_E_INVALID, "far-field kernel: missing source data");
    if (prof && prof->on) {
        PairProfiler::Rec r{prof_take_event(prof), prof_take_event(prof),
                            14 + 2 * J.cls + (J.prec == VSIE_FP32 ? 1 : 0),
                            static_cast<double>(J.n_d) * J.n_s, static_cast<double>(J.n_d) * J.n_s * J.nrhs};
        VSIE_HIP(hipEventRecord(r.a, s));
        launch_far_field(J, s, nullptr);
        VSIE_HIP(hipEventRecord(r.b, s));
        prof->recs.push_back(r);
        return;
    }
    if (J.cls == kClassG) run_far<kClassG>(J, s);
    else run_far<kClassF>(J, s);
}

}  // namespace vsie
