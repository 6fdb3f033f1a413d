// Product with the assembled FP32 operator (the dense block system of
// section 2.3.4 written once to memory) on the matrix cores of gfx950:
//   forward  y = d x + A x,      adjoint  y = conj(d) x + A^H x,
// for up to kDenseCols right-hand sides per pass.  A is stored as two
// column-major FP32 planes (real parts Ar, imaginary parts Ai, leading
// dimension ld); x and y are complex128.
//
// One work item is a 128 x 128 block of the output (rows: targets, columns:
// right-hand sides) over one slab of kDenseSlab sources.  Its four waves each
// own a 64 x 64 sub-block as 4 x 4 tiles of v_mfma_f32_16x16x4_f32.  The
// complex multiply-add uses three real products,
//   P1 = Ar Xr,  P2 = Ai Xi,  P3 = (Ar + Ai)(Xr + Xi),
//   Re = P1 - P2,  Im = P3 - P1 - P2,
// each in its own FP32 accumulator (or, without M3, the four products
// Ar Xr, Ai (-Xi), Ar Xi, Ai Xr).  Stages of 16 sources of both operands are
// staged in LDS, double-buffered: the global loads of stage s + 1 are in
// flight while stage s runs on the matrix cores.  At the end of the slab the
// FP32 sums are combined in FP64 and written as one FP64 partial per (slab,
// column, row); the reduction kernel adds the diagonal term and the slab
// partials in slab order (deterministic).
//
// The right-hand sides are packed once per pass to FP32 planes
// Xp[plane][j][c] (plane 0 real, 1 imaginary; c < 128, zero past nrhs and
// past n), so every stage reads 16 x 128 contiguous floats per plane.
#include "vsie_internal.h"

namespace vsie {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

constexpr int kXcds = 8;
constexpr int kTileM = 128;            // output rows per work item
constexpr int kTileN = kDenseCols;     // output columns per work item
constexpr int kStageK = 16;            // sources per LDS stage
constexpr int kLdsRow = kTileM + 16;   // floats per LDS row: conflict-free operand reads
constexpr int kLdsRowT = kStageK + 1;  // adjoint layout: floats per LDS row (one target)
constexpr int kStageFloats = 2 * kStageK * kLdsRow;  // one operand, both planes
static_assert(kTileN == kTileM, "square output tiles");
static_assert(2 * kTileM * kLdsRowT <= kStageFloats, "adjoint tile fits the stage");

struct DenseArgs {
    const float *__restrict__ ar;   // real plane
    const float *__restrict__ ai;   // imaginary plane
    int64_t ld;
    int64_t n;
    const float *__restrict__ xp;   // packed right-hand sides [2][npad][kTileN]
    int64_t npad;
    double2 *__restrict__ part;     // part[(s * nrhs + c) * n + i]
    int nrhs;
    int n_mt;                       // output row tiles
    int n_slabs;
    int64_t items;
};

// One stage in registers: per thread 16 values of A and 16 packed
// right-hand-side values.
//
// Forward: wave w loads columns 4w .. 4w + 3 of the stage in both planes,
// 128 rows each as two dword loads per lane (rows lane and 64 + lane): the
// column's base address is wave-uniform (scalar), the lane's offsets are
// fixed for the whole item, so the loads need no vector arithmetic.  Rows
// past n (the last row tile only) read row n - 1 instead: their products land
// in output rows that are never written.  Sources past n (the last stage of
// the last slab only) read column n - 1: finite values that meet the zero
// rows of the packed right-hand sides.  No load result is masked, so nothing
// waits for a load before the stage is written to LDS.
//
// Adjoint (A^H: output rows are columns of A, sources are rows of A): thread
// t loads four consecutive sources of one output row, clamped the same way.
//
// Packed right-hand sides: wave w loads rows 4w .. 4w + 3 of the stage in both
// planes, 128 columns each as one 8-byte load per lane.
struct StageRegs {
    float a[16];
    v2f x[8];
};

template <bool ADJ>
__device__ inline void load_stage(const DenseArgs &a, int wid, int lane, const int (&roff)[2], int64_t i0, int64_t k0,
                                  StageRegs &r) {
    const int64_t nm1 = a.n - 1;
    if constexpr (!ADJ) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int pl = c >> 2, kk = 4 * wid + (c & 3);
            int64_t j = k0 + kk;
            j = j < nm1 ? j : nm1;
            const float *__restrict__ col = (pl ? a.ai : a.ar) + j * a.ld + i0;
            r.a[2 * c] = col[roff[0]];
            r.a[2 * c + 1] = col[roff[1]];
        }
    } else {
        const int t = threadIdx.x;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = t + 256 * u;
            const int pl = q >> 9, m = (q >> 2) & 127, k4 = q & 3;
            int64_t jc = i0 + m;
            jc = jc < nm1 ? jc : nm1;
            const float *__restrict__ col = (pl ? a.ai : a.ar) + jc * a.ld;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int64_t ir = k0 + 4 * k4 + e;
                ir = ir < nm1 ? ir : nm1;
                r.a[4 * u + e] = col[ir];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int pl = c >> 2, kk = 4 * wid + (c & 3);
        // rows past n are zero in the packing (npad)
        r.x[c] = *reinterpret_cast<const v2f *>(a.xp + (pl * a.npad + k0 + kk) * kTileN + 2 * lane);
    }
}

// A stage from registers into LDS.  Operand A: [plane][source][row], row
// stride kLdsRow (forward), or [plane][row][source], stride kLdsRowT
// (adjoint).  Right-hand sides: [plane][source][column], stride kLdsRow.
template <bool ADJ>
__device__ inline void store_stage(float *__restrict__ la, float *__restrict__ lx, int wid, int lane,
                                   const StageRegs &r) {
    if constexpr (!ADJ) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int pl = c >> 2, kk = 4 * wid + (c & 3);
            float *__restrict__ d = la + (pl * kStageK + kk) * kLdsRow;
            d[lane] = r.a[2 * c];
            d[64 + lane] = r.a[2 * c + 1];
        }
    } else {
        const int t = threadIdx.x;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = t + 256 * u;
            const int pl = q >> 9, m = (q >> 2) & 127, k4 = q & 3;
            float *__restrict__ d = la + (pl * kTileM + m) * kLdsRowT + 4 * k4;
#pragma unroll
            for (int e = 0; e < 4; ++e) d[e] = r.a[4 * u + e];
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int pl = c >> 2, kk = 4 * wid + (c & 3);
        *reinterpret_cast<v2f *>(lx + (pl * kStageK + kk) * kLdsRow + 2 * lane) = r.x[c];
    }
}

template <bool ADJ, bool M3>
__global__ __launch_bounds__(256) void dense_cgemm_kernel(DenseArgs a) {
    __shared__ float lds[2][2 * kStageFloats];  // two stages of (A, X)
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int wm = wid >> 1, wn = wid & 1;  // 64 x 64 sub-block of the wave
    const int l16 = lane & 15, lq = lane >> 4;

    // item of this workgroup: contiguous ranges per XCD, slab-major so that
    // the waves of an XCD share one slab of packed right-hand sides
    const int xcd = blockIdx.x % kXcds;
    const int64_t per = (a.items + kXcds - 1) / kXcds;
    const int64_t item = xcd * per + blockIdx.x / kXcds;
    if (item >= a.items || blockIdx.x / kXcds >= per) return;
    const int s = static_cast<int>(item / a.n_mt);
    const int mt = static_cast<int>(item % a.n_mt);
    const int64_t i0 = static_cast<int64_t>(mt) * kTileM;
    const int64_t kbeg = static_cast<int64_t>(s) * kDenseSlab;
    const int64_t kend = (kbeg + kDenseSlab < a.n) ? kbeg + kDenseSlab : a.n;
    const int nst = static_cast<int>((kend - kbeg + kStageK - 1) / kStageK);
    // forward row offsets of this lane within the tile, clamped to row n - 1
    int roff[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t i = i0 + 64 * h + lane;
        roff[h] = static_cast<int>((i < a.n ? i : a.n - 1) - i0);
    }

    v4f d0[4][4], d1[4][4], d2[4][4], d3[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) d0[mb][nb] = d1[mb][nb] = d2[mb][nb] = d3[mb][nb] = v4f{0.f, 0.f, 0.f, 0.f};

    StageRegs r;
    load_stage<ADJ>(a, wid, lane, roff, i0, kbeg, r);
    store_stage<ADJ>(lds[0], lds[0] + kStageFloats, wid, lane, r);
    __syncthreads();

    for (int st = 0; st < nst; ++st) {
        if (st + 1 < nst) load_stage<ADJ>(a, wid, lane, roff, i0, kbeg + static_cast<int64_t>(st + 1) * kStageK, r);
        const float *__restrict__ la = lds[st & 1];
        const float *__restrict__ lx = la + kStageFloats;
#pragma unroll
        for (int ks = 0; ks < kStageK / 4; ++ks) {
            const int kk = 4 * ks + lq;
            float ar[4], ai[4], xr[4], xi[4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const int m = 64 * wm + 16 * mb + l16;
                if constexpr (!ADJ) {
                    ar[mb] = la[kk * kLdsRow + m];
                    ai[mb] = la[(kStageK + kk) * kLdsRow + m];
                } else {
                    ar[mb] = la[m * kLdsRowT + kk];
                    ai[mb] = la[(kTileM + m) * kLdsRowT + kk];
                }
            }
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const int c = 64 * wn + 16 * nb + l16;
                xr[nb] = lx[kk * kLdsRow + c];
                xi[nb] = lx[(kStageK + kk) * kLdsRow + c];
            }
            if constexpr (M3) {
                // A^H has -Ai: the third product takes (Ar - Ai); the signs of
                // the combination follow below
                float as[4], xs[4];
#pragma unroll
                for (int mb = 0; mb < 4; ++mb) as[mb] = ADJ ? ar[mb] - ai[mb] : ar[mb] + ai[mb];
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) xs[nb] = xr[nb] + xi[nb];
#pragma unroll
                for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb) {
                        d0[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[mb], xr[nb], d0[mb][nb], 0, 0, 0);
                        d1[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[mb], xi[nb], d1[mb][nb], 0, 0, 0);
                        d2[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[mb], xs[nb], d2[mb][nb], 0, 0, 0);
                    }
            } else {
                float xn[4];
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) xn[nb] = -xi[nb];
#pragma unroll
                for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb) {
                        d0[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[mb], xr[nb], d0[mb][nb], 0, 0, 0);
                        d1[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[mb], xn[nb], d1[mb][nb], 0, 0, 0);
                        d2[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[mb], xi[nb], d2[mb][nb], 0, 0, 0);
                        d3[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[mb], xr[nb], d3[mb][nb], 0, 0, 0);
                    }
            }
        }
        if (st + 1 < nst) {
            // the other buffer was last read in stage st - 1, which every wave
            // finished before the barrier that ended it
            float *__restrict__ wa = lds[(st + 1) & 1];
            store_stage<ADJ>(wa, wa + kStageFloats, wid, lane, r);
        }
        __syncthreads();
    }

    // D operand: lane l, register v holds row 4 (l / 16) + v, column l % 16
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const int c = 64 * wn + 16 * nb + l16;
        if (c >= a.nrhs) continue;
        double2 *__restrict__ o = a.part + (static_cast<int64_t>(s) * a.nrhs + c) * a.n;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = i0 + 64 * wm + 16 * mb + 4 * lq + v;
                if (i >= a.n) continue;
                const double p0 = d0[mb][nb][v], p1 = d1[mb][nb][v], p2 = d2[mb][nb][v];
                // forward: P1 = Ar Xr, P2 = Ai Xi, P3 = (Ar + Ai)(Xr + Xi);
                // adjoint (Ai -> -Ai): P3 = (Ar - Ai)(Xr + Xi), Re = P1 + P2,
                // Im = P3 - P1 + P2.  Four products: Ar Xr, Ai (-Xi), Ar Xi, Ai Xr.
                double re, im;
                if constexpr (M3) {
                    re = ADJ ? p0 + p1 : p0 - p1;
                    im = ADJ ? p2 - p0 + p1 : p2 - p0 - p1;
                } else {
                    const double p3 = d3[mb][nb][v];
                    re = ADJ ? p0 - p1 : p0 + p1;
                    im = ADJ ? p2 - p3 : p2 + p3;
                }
                o[i] = make_double2(re, im);
            }
    }
}

// xp[(pl npad + j) kTileN + c] = (Re, Im) of x[c ldx + j] for c < nrhs and j < n, else 0
__global__ void dense_pack_kernel(int64_t n, int64_t npad, int nrhs, const double2 *__restrict__ x, int64_t ldx,
                                  float *__restrict__ xp) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= npad * kTileN) return;
    const int64_t j = e / kTileN;
    const int c = static_cast<int>(e - j * kTileN);
    float re = 0.f, im = 0.f;
    if (c < nrhs && j < n) {
        const double2 v = x[c * ldx + j];
        re = static_cast<float>(v.x);
        im = static_cast<float>(v.y);
    }
    xp[j * kTileN + c] = re;
    xp[(npad + j) * kTileN + c] = im;
}

// y[c ldy + i] = d_i x[c ldx + i] (conj(d_i) for the adjoint) + sum over slabs in order
__global__ void dense_reduce_kernel(int64_t n, int nrhs, int n_slabs, const double2 *__restrict__ part,
                                    const double2 *__restrict__ diag, bool adj, const double2 *__restrict__ x,
                                    int64_t ldx, double2 *__restrict__ y, int64_t ldy) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n) return;
    const double2 d = diag[i], xv = x[c * ldx + i];
    const double di = adj ? -d.y : d.y;
    double re = d.x * xv.x - di * xv.y, im = d.x * xv.y + di * xv.x;
    for (int s = 0; s < n_slabs; ++s) {
        const double2 p = part[(static_cast<int64_t>(s) * nrhs + c) * n + i];
        re += p.x;
        im += p.y;
    }
    y[c * ldy + i] = make_double2(re, im);
}

}  // namespace

int64_t dense_npad(int64_t n) { return (n + kStageK - 1) / kStageK * kStageK; }

void launch_dense_product(const DenseJob &J, hipStream_t s, PairProfiler *prof) {
    const int64_t n = J.n;
    const int64_t npad = dense_npad(n);
    const int nrhs = J.nrhs;
    if (nrhs < 1 || nrhs > kTileN) fail(VSIE_E_INVALID, "dense product: 1 to 128 columns per pass");
    {
        const int64_t tot = npad * kTileN;
        hipLaunchKernelGGL(dense_pack_kernel, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s, n, npad,
                           nrhs, J.x, J.ldx, J.xp);
        VSIE_HIP(hipGetLastError());
    }
    DenseArgs a{J.ar, J.ai, J.ld, n, J.xp, npad, J.part, nrhs, 0, 0, 0};
    a.n_mt = static_cast<int>((n + kTileM - 1) / kTileM);
    a.n_slabs = static_cast<int>((n + kDenseSlab - 1) / kDenseSlab);
    a.items = static_cast<int64_t>(a.n_mt) * a.n_slabs;
    const int64_t per = (a.items + kXcds - 1) / kXcds;
    const dim3 grid(static_cast<unsigned>(per * kXcds));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (prof && prof->on) {
        ev0 = prof_take_event(prof);
        ev1 = prof_take_event(prof);
        VSIE_HIP(hipEventRecord(ev0, s));
    }
    if (J.adjoint) {
        if (J.m3) hipLaunchKernelGGL((dense_cgemm_kernel<true, true>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((dense_cgemm_kernel<true, false>), grid, dim3(256), 0, s, a);
    } else {
        if (J.m3) hipLaunchKernelGGL((dense_cgemm_kernel<false, true>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((dense_cgemm_kernel<false, false>), grid, dim3(256), 0, s, a);
    }
    VSIE_HIP(hipGetLastError());
    if (ev1) {
        // profiler kind 20: pairs = n^2 matrix entries, rhs_pairs = n^2 nrhs complex multiply-adds
        VSIE_HIP(hipEventRecord(ev1, s));
        const double e2 = static_cast<double>(n) * static_cast<double>(n);
        prof->recs.push_back(PairProfiler::Rec{ev0, ev1, 20, e2, e2 * nrhs});
    }
    hipLaunchKernelGGL(dense_reduce_kernel, dim3(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(nrhs)),
                       dim3(256), 0, s, n, nrhs, a.n_slabs, J.part, J.diag, J.adjoint, J.x, J.ldx, J.y, J.ldy);
    VSIE_HIP(hipGetLastError());
}

}  // namespace vsie
