// FP32 forward pair sums on the matrix cores of gfx950, for blocks of
// right-hand sides and several frequencies in one launch.
//
// The forward product of one source class is a complex matrix product
//   Y(targets x rhs) = K(targets x sources) Q(sources x rhs)
// with K_ij = e_ij (class G, single layer) or e_ij (i k r - 1) q_ij (class F,
// T and K terms), e = exp(i k r)/r, q = d.v'_j / r^2, and Q the packed charges
// (paper: the midpoint rule applied to eq_vsie, as in the vector pair kernel).
// K is never stored: each lane evaluates one kernel value per step straight
// into the A operand of v_mfma_f32_16x16x4_f32, whose 64 lanes hold a
// 16 (targets) x 4 (sources) block, lane l = target l % 16, source l / 16.
// The charges of those 4 sources and 16 right-hand sides form the B operand
// (lane l = source l / 16, column l % 16), one coalesced 512-byte read.  Four
// real products make the complex one:
//   Yr += Kr Qr - Ki Qi,   Yi += Kr Qi + Ki Qr.
// The VALU cost per pair (FP64 distance and phase, FP32 amplitude, sin, cos)
// no longer grows with the number of right-hand sides: one kernel value
// serves 16 (or 32) columns, whose multiply-adds run on the matrix cores.
//
// Accumulation: FP32 inside the matrix core over sub-tiles of kSubTile
// sources, then added into FP64 registers; one FP64 partial per (frequency,
// column, chunk, target), summed in chunk order by the reduction kernel.
//
// Schedule: work items are (frequency, column block, source chunk, target
// tile) with the target tile fastest; the item list is cut into 8 contiguous
// ranges, one per XCD (workgroup b runs on XCD b mod 8), so the waves of one
// XCD walk neighbouring target tiles of the same source chunk and share its
// positions and charges in their L2.  Wave w of an XCD takes items w, w + W,
// ... of its range (W = waves per XCD); by default the grid gives every wave
// one item and the hardware dispatcher balances the load.
#include "pair_geom.h"
#include "vsie_internal.h"

namespace vsie {
namespace {

using namespace geom;

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kXcds = 8;
constexpr int kSubTile = 128;   // sources per FP32 accumulation
constexpr int kWavesPerBlock = kBlock / 64;

struct MfmaArgs {
    int64_t n_t;
    const double *__restrict__ tx;
    const double *__restrict__ ty;
    const double *__restrict__ tz;
    int64_t n_s;
    const double4 *__restrict__ pk;  // sources (x, y, z, 0), padded
    const double4 *__restrict__ pv;  // F: (v'x, v'y, v'z, 0), padded
    const float2 *__restrict__ q;    // q[fl * ldq_f + j * ncol + col], zero rows past n_s
    int64_t ldq_f;
    int ncol;
    int nrhs;
    const double *__restrict__ kf;   // k of each local frequency
    int64_t chunk;                   // a multiple of 4
    int n_chunks;
    int n_tiles;
    int n_cb;
    int64_t items;
    double2 *__restrict__ out;
    int64_t out_fstride;
    int part0;
};

template <int CLS, int TG, int NB, bool M3>
__global__ __launch_bounds__(kBlock) void mfma_fwd_kernel(MfmaArgs a) {
    constexpr int TT = 16 * TG;  // targets per item
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int xcd = blockIdx.x % kXcds;
    const int64_t waves_x = static_cast<int64_t>(gridDim.x / kXcds) * kWavesPerBlock;
    const int64_t w = static_cast<int64_t>(blockIdx.x / kXcds) * kWavesPerBlock + wib;
    const int64_t lo = a.items * xcd / kXcds, hi = a.items * (xcd + 1) / kXcds;
    const int tl = lane & 15;   // A operand: target row; B, D: column
    const int sq = lane >> 4;   // A, B operand: source row; D: row quad
    const uint32_t qrow = static_cast<uint32_t>(a.ncol) * 8u;  // bytes per source row of q

    for (int64_t it = lo + w; it < hi; it += waves_x) {
        int64_t t = it;
        const int tt = static_cast<int>(t % a.n_tiles);
        t /= a.n_tiles;
        const int c = static_cast<int>(t % a.n_chunks);
        t /= a.n_chunks;
        const int cb = static_cast<int>(t % a.n_cb);
        const int fl = static_cast<int>(t / a.n_cb);

        const double k = a.kf[fl];
        const float kf = static_cast<float>(k);
        const double kr2pi = k / kTwoPi;
        const int64_t ib = static_cast<int64_t>(tt) * TT;
        double xi[TG], yi[TG], zi[TG];
#pragma unroll
        for (int g = 0; g < TG; ++g) {
            int64_t i = ib + 16 * g + tl;
            i = i < a.n_t ? i : a.n_t - 1;
            xi[g] = a.tx[i];
            yi[g] = a.ty[i];
            zi[g] = a.tz[i];
        }
        const int64_t j0 = static_cast<int64_t>(c) * a.chunk;
        const int64_t j1 = (j0 + a.chunk < a.n_s) ? j0 + a.chunk : a.n_s;
        const char *__restrict__ pkb = reinterpret_cast<const char *>(a.pk);
        const char *__restrict__ pvb = reinterpret_cast<const char *>(a.pv);
        const char *__restrict__ qb = reinterpret_cast<const char *>(a.q + fl * a.ldq_f + cb * (16 * NB));

        double accr[TG][NB][4], acci[TG][NB][4];
#pragma unroll
        for (int g = 0; g < TG; ++g)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) accr[g][b][v] = acci[g][b][v] = 0.0;

        for (int64_t jt = j0; jt < j1; jt += kSubTile) {
            const int64_t je = (jt + kSubTile < j1) ? jt + kSubTile : j1;
            // steps of 4 sources; past n_s the padding (zero charges) is read
            const int steps = static_cast<int>((je - jt + 3) >> 2);
            uint32_t po = static_cast<uint32_t>(jt + sq) * 32u;
            uint32_t qo = static_cast<uint32_t>(jt + sq) * qrow + static_cast<uint32_t>(tl) * 8u;
            // one accumulator per real product, so that no two matrix-core
            // operations of a step depend on each other: Kr Qr, Ki (-Qi), Kr Qi,
            // Ki Qr; or, with M3, Kr Qr, Ki Qi, (Kr + Ki)(Qr + Qi), from which
            // Re = P1 - P2 and Im = P3 - P1 - P2 (three products instead of four)
            v4f d0[TG][NB], d1[TG][NB], d2[TG][NB], d3[TG][NB];
#pragma unroll
            for (int g = 0; g < TG; ++g)
#pragma unroll
                for (int b = 0; b < NB; ++b) d0[g][b] = d1[g][b] = d2[g][b] = d3[g][b] = v4f{0.f, 0.f, 0.f, 0.f};
            // software pipeline: the positions and charges of step st + 1 are in
            // flight while step st computes (the last prefetch reads at most 7
            // entries past n_s: inside the padding)
            double4 Pn = *reinterpret_cast<const double4 *>(pkb + po);
            double4 Vn = make_double4(0.0, 0.0, 0.0, 0.0);
            if constexpr (CLS == kClassF) Vn = *reinterpret_cast<const double4 *>(pvb + po);
            float2 un[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) un[b] = *reinterpret_cast<const float2 *>(qb + qo + 128u * b);
            for (int st = 0; st < steps; ++st) {
                const double4 P = Pn;
                const double4 Vv = Vn;
                float qr[NB], qi[NB], qn[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    qr[b] = un[b].x;
                    qi[b] = un[b].y;
                    qn[b] = M3 ? un[b].x + un[b].y : -un[b].y;
                }
                po += 128u;
                qo += 4u * qrow;
                Pn = *reinterpret_cast<const double4 *>(pkb + po);
                if constexpr (CLS == kClassF) Vn = *reinterpret_cast<const double4 *>(pvb + po);
#pragma unroll
                for (int b = 0; b < NB; ++b) un[b] = *reinterpret_cast<const float2 *>(qb + qo + 128u * b);
#pragma unroll
                for (int g = 0; g < TG; ++g) {
                    const double dx = xi[g] - P.x, dy = yi[g] - P.y, dz = zi[g] - P.z;
                    float er, ei, ir2, kr;
                    // every pair is masked: one loop body keeps the accumulators in place
                    geom_f32<true>(dx, dy, dz, kf, kr2pi, er, ei, ir2, kr);
                    float kre = er, kim = ei;
                    if constexpr (CLS == kClassF) {
                        const float qq = static_cast<float>(fma(dx, Vv.x, fma(dy, Vv.y, dz * Vv.z))) * ir2;
                        kre = qq * fmaf(-ei, kr, -er);
                        kim = qq * fmaf(er, kr, -ei);
                    }
                    if constexpr (M3) {
                        const float ks = kre + kim;
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            d0[g][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(kre, qr[b], d0[g][b], 0, 0, 0);
                            d1[g][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(kim, qi[b], d1[g][b], 0, 0, 0);
                            d2[g][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ks, qn[b], d2[g][b], 0, 0, 0);
                        }
                    } else {
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            d0[g][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(kre, qr[b], d0[g][b], 0, 0, 0);
                            d1[g][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(kim, qn[b], d1[g][b], 0, 0, 0);
                            d2[g][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(kre, qi[b], d2[g][b], 0, 0, 0);
                            d3[g][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(kim, qr[b], d3[g][b], 0, 0, 0);
                        }
                    }
                }
                // the prefetched values are live here: their loads stay inside this step
                asm volatile("" : "+v"(Pn.x), "+v"(Pn.y), "+v"(Pn.z));
                if constexpr (CLS == kClassF) asm volatile("" : "+v"(Vn.x), "+v"(Vn.y), "+v"(Vn.z));
#pragma unroll
                for (int b = 0; b < NB; ++b) asm volatile("" : "+v"(un[b].x), "+v"(un[b].y));
            }
#pragma unroll
            for (int g = 0; g < TG; ++g)
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double p0 = d0[g][b][v], p1 = d1[g][b][v], p2 = d2[g][b][v];
                        if constexpr (M3) {
                            accr[g][b][v] += p0 - p1;
                            acci[g][b][v] += p2 - p0 - p1;
                        } else {
                            accr[g][b][v] += p0 + p1;
                            acci[g][b][v] += p2 + static_cast<double>(d3[g][b][v]);
                        }
                    }
        }
        // D operand: lane l, register v holds target row 4 (l / 16) + v, column l % 16
        double2 *__restrict__ o = a.out + fl * a.out_fstride +
                                  static_cast<int64_t>(a.part0 + c) * a.nrhs * a.n_t;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int col = cb * (16 * NB) + 16 * b + tl;
            if (col >= a.nrhs) continue;
#pragma unroll
            for (int g = 0; g < TG; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t i = ib + 16 * g + 4 * sq + v;
                    if (i < a.n_t) o[static_cast<int64_t>(col) * a.n_t + i] = make_double2(accr[g][b][v], acci[g][b][v]);
                }
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 forward pair sums on the FP64 matrix cores (v_mfma_f64_16x16x4_f64):
// the same product Y = K Q as above with K evaluated in FP64 (geom_f64: FP64
// distance, phase and series sine and cosine) and FP64 charges, accumulated
// in FP64 by the matrix core over the whole source chunk.  One kernel
// evaluation per pair serves 16 NB columns; the VALU's FP64 multiply-adds per
// pair and column (four in the vector kernel) move to the matrix core, whose
// FP64 rate equals the VALU's, at three real products per complex one (M3)
// spread over 16 x 16 x 4 blocks.  Work items and XCD ranges as above; two
// 16-target groups per wave.
typedef double v4d __attribute__((ext_vector_type(4)));

struct Mfma64Args {
    int64_t n_t;
    const double *__restrict__ tx;
    const double *__restrict__ ty;
    const double *__restrict__ tz;
    int64_t n_s;
    const double4 *__restrict__ pk;
    const double4 *__restrict__ pv;
    const double2 *__restrict__ q;   // q[fl * ldq_f + j * ncol + col], zero rows past n_s
    int64_t ldq_f;
    int ncol;
    int nrhs;
    const double *__restrict__ kf;
    int64_t chunk;                    // a multiple of 4
    int n_chunks;
    int n_tiles;
    int n_cb;
    int64_t items;
    double2 *__restrict__ out;
    int64_t out_fstride;
    int part0;
};


template <int CLS, int NB, bool M3>
__global__ __launch_bounds__(kBlock) void mfma64_fwd_kernel(Mfma64Args a) {
    constexpr int TG = mfma64_groups(CLS, NB);
    constexpr int TT = 16 * TG;
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int xcd = blockIdx.x % kXcds;
    const int64_t waves_x = static_cast<int64_t>(gridDim.x / kXcds) * kWavesPerBlock;
    const int64_t w = static_cast<int64_t>(blockIdx.x / kXcds) * kWavesPerBlock + wib;
    const int64_t lo = a.items * xcd / kXcds, hi = a.items * (xcd + 1) / kXcds;
    const int tl = lane & 15, sq = lane >> 4;

    for (int64_t it = lo + w; it < hi; it += waves_x) {
        int64_t t = it;
        const int tt = static_cast<int>(t % a.n_tiles);
        t /= a.n_tiles;
        const int c = static_cast<int>(t % a.n_chunks);
        t /= a.n_chunks;
        const int cb = static_cast<int>(t % a.n_cb);
        const int fl = static_cast<int>(t / a.n_cb);
        const double k = a.kf[fl];
        const double khalf = k / kPi;
        const int64_t ib = static_cast<int64_t>(tt) * TT;
        double xi[TG], yi[TG], zi[TG];
#pragma unroll
        for (int g = 0; g < TG; ++g) {
            int64_t i = ib + 16 * g + tl;
            i = i < a.n_t ? i : a.n_t - 1;
            xi[g] = a.tx[i];
            yi[g] = a.ty[i];
            zi[g] = a.tz[i];
        }
        const int64_t j0 = static_cast<int64_t>(c) * a.chunk;
        const int64_t j1 = (j0 + a.chunk < a.n_s) ? j0 + a.chunk : a.n_s;
        const double2 *__restrict__ qb = a.q + fl * a.ldq_f + cb * (16 * NB);
        v4d d0[TG][NB], d1[TG][NB], d2[TG][NB], d3[TG][NB];
#pragma unroll
        for (int g = 0; g < TG; ++g)
#pragma unroll
            for (int b = 0; b < NB; ++b) d0[g][b] = d1[g][b] = d2[g][b] = d3[g][b] = v4d{0.0, 0.0, 0.0, 0.0};
        // steps of 4 sources; past n_s the padding (far points, zero charges) is
        // read.  Software pipeline: the positions and charges of step st + 1
        // are in flight while step st computes (the last prefetch reads at
        // most 7 entries past n_s: inside the padding).
        const int steps = static_cast<int>((j1 - j0 + 3) >> 2);
        int64_t jn = j0 + sq;
        double4 Pn = a.pk[jn];
        double4 Vn = make_double4(0.0, 0.0, 0.0, 0.0);
        if constexpr (CLS == kClassF) Vn = a.pv[jn];
        double2 un[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) un[b] = qb[jn * a.ncol + 16 * b + tl];
        for (int st = 0; st < steps; ++st) {
            const double4 P = Pn;
            const double4 Vv = Vn;
            double qr[NB], qi[NB], qn[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                qr[b] = un[b].x;
                qi[b] = un[b].y;
                qn[b] = M3 ? un[b].x + un[b].y : -un[b].y;
            }
            jn += 4;
            Pn = a.pk[jn];
            if constexpr (CLS == kClassF) Vn = a.pv[jn];
#pragma unroll
            for (int b = 0; b < NB; ++b) un[b] = qb[jn * a.ncol + 16 * b + tl];
#pragma unroll
            for (int g = 0; g < TG; ++g) {
                const double dx = xi[g] - P.x, dy = yi[g] - P.y, dz = zi[g] - P.z;
                double er, ei, ir2, kr;
                geom_f64<true>(dx, dy, dz, k, khalf, er, ei, ir2, kr);
                double kre = er, kim = ei;
                if constexpr (CLS == kClassF) {
                    const double qq = fma(dx, Vv.x, fma(dy, Vv.y, dz * Vv.z)) * ir2;
                    kre = qq * fma(-ei, kr, -er);
                    kim = qq * fma(er, kr, -ei);
                }
                if constexpr (M3) {
                    const double ks = kre + kim;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        d0[g][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kre, qr[b], d0[g][b], 0, 0, 0);
                        d1[g][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kim, qi[b], d1[g][b], 0, 0, 0);
                        d2[g][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ks, qn[b], d2[g][b], 0, 0, 0);
                    }
                } else {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        d0[g][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kre, qr[b], d0[g][b], 0, 0, 0);
                        d1[g][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kim, qn[b], d1[g][b], 0, 0, 0);
                        d2[g][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kre, qi[b], d2[g][b], 0, 0, 0);
                        d3[g][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kim, qr[b], d3[g][b], 0, 0, 0);
                    }
                }
            }
            // the prefetched values are live here: their loads stay inside this step
            asm volatile("" : "+v"(Pn.x), "+v"(Pn.y), "+v"(Pn.z));
            if constexpr (CLS == kClassF) asm volatile("" : "+v"(Vn.x), "+v"(Vn.y), "+v"(Vn.z));
#pragma unroll
            for (int b = 0; b < NB; ++b) asm volatile("" : "+v"(un[b].x), "+v"(un[b].y));
        }
        // D operand of the FP64 instruction: lane l, register v holds target row
        // 4 v + l / 16, column l % 16 (checked on the device with an in-bounds
        // one-hot probe; the FP32 instruction has row 4 (l / 16) + v)
        double2 *__restrict__ o = a.out + fl * a.out_fstride + static_cast<int64_t>(a.part0 + c) * a.nrhs * a.n_t;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int col = cb * (16 * NB) + 16 * b + tl;
            if (col >= a.nrhs) continue;
#pragma unroll
            for (int g = 0; g < TG; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t i = ib + 16 * g + 4 * v + sq;
                    if (i >= a.n_t) continue;
                    double re, im;
                    if constexpr (M3) {
                        re = d0[g][b][v] - d1[g][b][v];
                        im = d2[g][b][v] - d0[g][b][v] - d1[g][b][v];
                    } else {
                        re = d0[g][b][v] + d1[g][b][v];
                        im = d2[g][b][v] + d3[g][b][v];
                    }
                    o[static_cast<int64_t>(col) * a.n_t + i] = make_double2(re, im);
                }
        }
    }
}

// q[fl * ldq_f + jj * ncol + col] = scale * x[fl * xfs + col * ldx + idx[jj]] in FP64 (else as pack_mfma_kernel)
__global__ void pack_mfma64_kernel(int64_t count, const int32_t *__restrict__ idx, const double *__restrict__ sp,
                                   int64_t sp_fstride, int nrhs, int ncol, const double2 *__restrict__ x,
                                   int64_t ldx, int64_t xfs, double2 *__restrict__ q, int64_t ldq_f) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int fl = blockIdx.y;
    if (e >= (count + kMfmaPad) * ncol) return;
    const int64_t jj = e / ncol;
    const int col = static_cast<int>(e - jj * ncol);
    double2 v = make_double2(0.0, 0.0);
    if (col < nrhs && jj < count) {
        const int64_t g = idx[jj];
        const double2 xv = x[fl * xfs + col * ldx + g];
        const double sc = sp ? -sp[fl * sp_fstride + g] : 1.0;
        v = make_double2(sc * xv.x, sc * xv.y);
    }
    q[fl * ldq_f + e] = v;
}

template <int CLS, int NB, bool M3>
const void *kernel64_ptr() {
    return reinterpret_cast<const void *>(&mfma64_fwd_kernel<CLS, NB, M3>);
}

template <bool M3>
const void *pick64_variant(int cls, int nb) {
    if (cls == kClassG) {
        if (nb == 1) return kernel64_ptr<kClassG, 1, M3>();
        if (nb == 2) return kernel64_ptr<kClassG, 2, M3>();
        if (nb == 4) return kernel64_ptr<kClassG, 4, M3>();
    } else {
        if (nb == 1) return kernel64_ptr<kClassF, 1, M3>();
        if (nb == 2) return kernel64_ptr<kClassF, 2, M3>();
        if (nb == 4) return kernel64_ptr<kClassF, 4, M3>();
    }
    return nullptr;
}

// q[fl * ldq_f + jj * ncol + col] = scale * x[fl * xfs + col * ldx + idx[jj]], 0 for col >= nrhs
// and for the kMfmaPad padding rows jj >= count; scale = -s'_f[idx[jj]] for class G, else 1
__global__ void pack_mfma_kernel(int64_t count, const int32_t *__restrict__ idx, const double *__restrict__ sp,
                                 int64_t sp_fstride, int nrhs, int ncol, const double2 *__restrict__ x,
                                 int64_t ldx, int64_t xfs, float2 *__restrict__ q, int64_t ldq_f) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int fl = blockIdx.y;
    if (e >= (count + kMfmaPad) * ncol) return;
    const int64_t jj = e / ncol;
    const int col = static_cast<int>(e - jj * ncol);
    float2 v = make_float2(0.f, 0.f);
    if (col < nrhs && jj < count) {
        const int64_t g = idx[jj];
        const double2 xv = x[fl * xfs + col * ldx + g];
        const double sc = sp ? -sp[fl * sp_fstride + g] : 1.0;
        v = make_float2(static_cast<float>(sc * xv.x), static_cast<float>(sc * xv.y));
    }
    q[fl * ldq_f + e] = v;
}

template <int CLS, int TG, int NB, bool M3>
const void *kernel_ptr() {
    return reinterpret_cast<const void *>(&mfma_fwd_kernel<CLS, TG, NB, M3>);
}

template <bool M3>
const void *pick_variant(int cls, int tg, int nb) {
    if (cls == kClassG) {
        if (tg == 4 && nb == 1) return kernel_ptr<kClassG, 4, 1, M3>();
        if (tg == 2 && nb == 1) return kernel_ptr<kClassG, 2, 1, M3>();
        if (tg == 2 && nb == 2) return kernel_ptr<kClassG, 2, 2, M3>();
        if (tg == 4 && nb == 2) return kernel_ptr<kClassG, 4, 2, M3>();
    } else {
        if (tg == 4 && nb == 1) return kernel_ptr<kClassF, 4, 1, M3>();
        if (tg == 2 && nb == 1) return kernel_ptr<kClassF, 2, 1, M3>();
        if (tg == 2 && nb == 2) return kernel_ptr<kClassF, 2, 2, M3>();
        if (tg == 4 && nb == 2) return kernel_ptr<kClassF, 4, 2, M3>();
    }
    return nullptr;
}

const void *pick_kernel(int cls, int tg, int nb, bool m3) {
    return m3 ? pick_variant<true>(cls, tg, nb) : pick_variant<false>(cls, tg, nb);
}

}  // namespace

bool mfma_variant_ok(int tg, int nb) { return pick_kernel(kClassG, tg, nb, false) != nullptr; }

int mfma_grid(int tg, int nb) {
    static int cus = 0;
    static int occ[2][2][2] = {};
    if (!cus) {
        int dev = 0;
        VSIE_HIP(hipGetDevice(&dev));
        VSIE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    }
    const int ti = tg == 4 ? 1 : 0, bi = nb == 2 ? 1 : 0;
    int &o = occ[0][ti][bi];
    if (!o) {
        int og = 0, of = 0;
        VSIE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&og, pick_kernel(kClassG, tg, nb, false), kBlock, 0));
        VSIE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&of, pick_kernel(kClassF, tg, nb, false), kBlock, 0));
        o = std::max(1, std::min(og, of));
    }
    const int g = cus * o;
    return std::max(kXcds, (g / kXcds) * kXcds);
}

void launch_pack_mfma(SrcClass cls, const SourceSet &src, const double *sp, int64_t sp_fstride, int nf,
                      int nrhs, int ncol, const double2 *x, int64_t ldx, int64_t xfs, float2 *q, int64_t ldq_f,
                      hipStream_t s) {
    if (src.count == 0 || nf == 0) return;
    if (ldq_f < (src.count + kMfmaPad) * ncol) fail(VSIE_E_INVALID, "matrix-core charges: stride too small");
    const int64_t total = (src.count + kMfmaPad) * ncol;
    dim3 grid(static_cast<unsigned>((total + kBlock - 1) / kBlock), static_cast<unsigned>(nf));
    hipLaunchKernelGGL(pack_mfma_kernel, grid, dim3(kBlock), 0, s, src.count, src.idx,
                       cls == kClassG ? sp : nullptr, sp_fstride, nrhs, ncol, x, ldx, xfs, q, ldq_f);
    VSIE_HIP(hipGetLastError());
}

void launch_pack_mfma64(SrcClass cls, const SourceSet &src, const double *sp, int64_t sp_fstride, int nf,
                        int nrhs, int ncol, const double2 *x, int64_t ldx, int64_t xfs, double2 *q, int64_t ldq_f,
                        hipStream_t s) {
    if (src.count == 0 || nf == 0) return;
    if (ldq_f < (src.count + kMfmaPad) * ncol) fail(VSIE_E_INVALID, "FP64 matrix-core charges: stride too small");
    const int64_t total = (src.count + kMfmaPad) * ncol;
    dim3 grid(static_cast<unsigned>((total + kBlock - 1) / kBlock), static_cast<unsigned>(nf));
    hipLaunchKernelGGL(pack_mfma64_kernel, grid, dim3(kBlock), 0, s, src.count, src.idx,
                       cls == kClassG ? sp : nullptr, sp_fstride, nrhs, ncol, x, ldx, xfs, q, ldq_f);
    VSIE_HIP(hipGetLastError());
}

bool mfma64_nb_ok(int nb) { return nb == 1 || nb == 2 || nb == 4; }

void launch_mfma64_forward(const Mfma64Job &J, hipStream_t s, PairProfiler *prof) {
    if (J.n_t == 0 || J.n_s == 0 || J.nf == 0) return;
    const int TT = 16 * mfma64_groups(J.cls, J.nb);
    const int cbw = 16 * J.nb;
    if (!mfma64_nb_ok(J.nb)) fail(VSIE_E_INVALID, "FP64 matrix-core pair kernel: unsupported column blocking");
    if (J.ncol % cbw != 0 || J.ncol < J.nrhs || J.nrhs <= 0)
        fail(VSIE_E_INVALID, "FP64 matrix-core pair kernel: inconsistent column blocking");
    if (J.chunk <= 0 || J.chunk % 4 != 0 || J.n_chunks <= 0 || (J.n_chunks - 1) * J.chunk >= J.n_s)
        fail(VSIE_E_INVALID, "FP64 matrix-core pair kernel: inconsistent source chunking");
    if (J.ldq_f < (J.n_s + kMfmaPad) * J.ncol)
        fail(VSIE_E_INVALID, "FP64 matrix-core pair kernel: charge block too small");
    if (!J.pk || (J.cls == kClassF && !J.pv))
        fail(VSIE_E_INVALID, "FP64 matrix-core pair kernel: source layout missing");
    Mfma64Args a{};
    a.n_t = J.n_t;
    a.tx = J.tx;
    a.ty = J.ty;
    a.tz = J.tz;
    a.n_s = J.n_s;
    a.pk = J.pk;
    a.pv = J.pv;
    a.q = J.q;
    a.ldq_f = J.ldq_f;
    a.ncol = J.ncol;
    a.nrhs = J.nrhs;
    a.kf = J.kf;
    a.chunk = J.chunk;
    a.n_chunks = J.n_chunks;
    a.n_tiles = static_cast<int>((J.n_t + TT - 1) / TT);
    a.n_cb = J.ncol / cbw;
    a.items = static_cast<int64_t>(J.nf) * a.n_cb * a.n_chunks * a.n_tiles;
    a.out = J.out;
    a.out_fstride = J.out_fstride;
    a.part0 = J.part0;
    const int64_t grid = one_item_per_wave_grid(a.items);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (prof && prof->on) {
        ev0 = prof_take_event(prof);
        ev1 = prof_take_event(prof);
        VSIE_HIP(hipEventRecord(ev0, s));
    }
    const void *kp = J.m3 ? pick64_variant<true>(J.cls, J.nb) : pick64_variant<false>(J.cls, J.nb);
    hipLaunchKernelGGL(reinterpret_cast<void (*)(Mfma64Args)>(const_cast<void *>(kp)), dim3(static_cast<unsigned>(grid)),
                       dim3(kBlock), 0, s, a);
    VSIE_HIP(hipGetLastError());
    if (prof && prof->on) {
        VSIE_HIP(hipEventRecord(ev1, s));
        const double pairs = static_cast<double>(J.n_t) * J.n_s * J.nf;
        // kinds 21 and 22: the FP64 matrix-core single layer and double layers
        prof->recs.push_back(PairProfiler::Rec{ev0, ev1, 21 + J.cls, pairs, pairs * J.nrhs});
    }
}

void launch_mfma_forward(const MfmaJob &J, hipStream_t s, PairProfiler *prof) {
    if (J.n_t == 0 || J.n_s == 0 || J.nf == 0) return;
    const int TT = 16 * J.tg;
    const int cbw = 16 * J.nb;
    if (!mfma_variant_ok(J.tg, J.nb)) fail(VSIE_E_INVALID, "matrix-core pair kernel: unsupported variant");
    if (J.ncol % cbw != 0 || J.ncol < J.nrhs || J.nrhs <= 0)
        fail(VSIE_E_INVALID, "matrix-core pair kernel: inconsistent column blocking");
    if (J.chunk <= 0 || J.chunk % 4 != 0 || J.n_chunks <= 0 || (J.n_chunks - 1) * J.chunk >= J.n_s)
        fail(VSIE_E_INVALID, "matrix-core pair kernel: inconsistent source chunking");
    if (J.ldq_f < (J.n_s + kMfmaPad) * J.ncol || (J.n_s + kMfmaPad) * J.ncol * 8 >= (int64_t(1) << 32))
        fail(VSIE_E_INVALID, "matrix-core pair kernel: charge block too small or above 4 GiB");
    if (!J.pk || (J.cls == kClassF && !J.pv))
        fail(VSIE_E_INVALID, "matrix-core pair kernel: source layout missing");
    MfmaArgs a{};
    a.n_t = J.n_t;
    a.tx = J.tx;
    a.ty = J.ty;
    a.tz = J.tz;
    a.n_s = J.n_s;
    a.pk = J.pk;
    a.pv = J.pv;
    a.q = J.q;
    a.ldq_f = J.ldq_f;
    a.ncol = J.ncol;
    a.nrhs = J.nrhs;
    a.kf = J.kf;
    a.chunk = J.chunk;
    a.n_chunks = J.n_chunks;
    a.n_tiles = static_cast<int>((J.n_t + TT - 1) / TT);
    a.n_cb = J.ncol / cbw;
    a.items = static_cast<int64_t>(J.nf) * a.n_cb * a.n_chunks * a.n_tiles;
    a.out = J.out;
    a.out_fstride = J.out_fstride;
    a.part0 = J.part0;
    const int64_t grid = J.grid > 0 ? J.grid : one_item_per_wave_grid(a.items);
    if (grid % kXcds != 0) fail(VSIE_E_INVALID, "matrix-core pair kernel: grid must be a multiple of 8");
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (prof && prof->on) {
        ev0 = prof_take_event(prof);
        ev1 = prof_take_event(prof);
        VSIE_HIP(hipEventRecord(ev0, s));
    }
    hipLaunchKernelGGL(reinterpret_cast<void (*)(MfmaArgs)>(const_cast<void *>(pick_kernel(J.cls, J.tg, J.nb, J.m3))),
                       dim3(static_cast<unsigned>(grid)), dim3(kBlock), 0, s, a);
    VSIE_HIP(hipGetLastError());
    if (prof && prof->on) {
        VSIE_HIP(hipEventRecord(ev1, s));
        const double pairs = static_cast<double>(J.n_t) * J.n_s * J.nf;
        prof->recs.push_back(PairProfiler::Rec{ev0, ev1, 8 + J.cls, pairs, pairs * J.nrhs});
    }
}

}  // namespace vsie
