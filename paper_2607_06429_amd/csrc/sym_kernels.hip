// Single-layer sums between volume cells, one kernel evaluation per
// unordered pair (one right-hand side).
//
// The single-layer term of the operator pairs every cell i with every cell j
// through e_ij = exp(i k r)/r, which is symmetric (paper: the midpoint rule
// applied to eq_vsie; G(r) depends on |x_i - y_j| only).  With charges
// u_j = -s'_j x_j the two contributions of a pair are
//   y_i += e_ij u_j   and   y_j += e_ij u_i,
// so one evaluation of e_ij (the FP64 distance and phase and the sine and
// cosine, which dominate the cost) serves both.
//
// Lanes and rotation: a wave pairs a 64-point tile A with a 64-point tile B.
// Lane l keeps point a_l (position, charge, accumulator).  In step k it meets
// B point (l - k) mod 64: the B positions and charges sit in the wave's own
// LDS slice (written once per tile pair; the LDS executes one wave's
// operations in order, so no barrier is needed), and the B point's
// source-side accumulator moves one lane along the wave after every step
// (DPP wavefront rotate).  After 64 steps each B accumulator is back in its
// home lane: both sides are lane-local, with no cross-lane reduction and no
// atomics.  A tile paired with itself runs 63 steps with the target side
// only.
//
// Work: the tiles are grouped G at a time.  A work item is a pair of groups
// (I, J), I <= J, and covers every tile pair between them (for I = J the
// tile pairs ta <= tb).  The points of group I receive their partial sum
// from the item in slot J and the points of group J in slot I, so every cell
// gets exactly one partial per group: part[slot * ldp + p].  A reduction
// kernel adds them in slot order (deterministic).
//
// With the adjoint double layer (T, cells with grad alpha, v'_i != 0) the
// same evaluation also gives F = e (i k r - 1)/r^2 and both directions of
// that term, q x with q = (x_target - y_source).v'_source:
//   y_i += F (d.v'_j) x_j   and   y_j += F (-d.v'_i) x_i,   d = x_i - x_j.
// Items whose tiles hold no such cell run the single-layer loop alone.
//
// The adjoint variant (with T) takes charges mu = conj(lambda) and puts the
// weights on the target side, (A^H)_ji = conj(A_ij):
//   z_i += (-s'_i e + F (-d.v'_i)) mu_j   and   z_j += (-s'_j e + F (d.v'_j)) mu_i;
// items without grad-alpha cells sum e mu and scale by -s' per tile pair.
//
// Schedule: items cut into 8 contiguous ranges (one per XCD, workgroup b
// runs on XCD b mod 8), one item per wave, so that the hardware dispatcher
// balances the load within an XCD.  The ranges hold equal modelled work: an
// item with grad-alpha cells counts as its issue cycles per pair relative to
// a single-layer item (the host computes the boundaries).  (A persistent grid with a static split leaves the tail
// to a few waves: the SIMD issues to its oldest wave first, so waves finish
// one by one and the last wave on each SIMD runs nearly alone.)
#include <type_traits>

#include "pair_geom.h"
#include "vsie_internal.h"

namespace vsie {
namespace {

using namespace geom;

constexpr int kXcds = 8;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kDppWaveRor1 = 0x13C;  // DPP control: rotate the whole wave right by one lane

// every lane has a source lane under a whole-wave rotate, so no "old" value is needed
__device__ __forceinline__ float rot1(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), kDppWaveRor1, 0xF, 0xF, true));
}
__device__ __forceinline__ double rot1(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(b), kDppWaveRor1, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(b >> 32), kDppWaveRor1, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

template <typename AT> struct c2_of;
template <> struct c2_of<double> { using type = double2; };
template <> struct c2_of<float> { using type = float2; };

struct SymArgs {
    int64_t ng;                     // cells (canonical points 0 .. ng-1)
    const double *__restrict__ px;
    const double *__restrict__ py;
    const double *__restrict__ pz;
    const void *__restrict__ q;     // charges u, complex AT, ng entries
    double k;
    double kphase;                  // k/pi (FP64: half turns) or k/(2 pi) (FP32: turns)
    double far[3];                  // padding position, farther than the mesh extent from every point
    double far_step;                // distance between padding positions
    int tiles;
    int groups;
    int64_t items;
    int64_t xr[kXcds + 1];           // item range of XCD x: [xr[x], xr[x + 1])
    void *__restrict__ part;         // slot partials: float2 (FP32 kernels) or double2
    int64_t ldp;
    // adjoint double layer (T variant only): v' of the cells, the raw values
    // x, and per 64-cell tile whether any v' is nonzero
    const double *__restrict__ vx;
    const double *__restrict__ vy;
    const double *__restrict__ vz;
    const double2 *__restrict__ xv;
    const int32_t *__restrict__ tile_t;
    const double *__restrict__ sw;  // adjoint variant: s' of the cells for this frequency
};

// position and charge of point p of a tile (padding lanes: distinct far points, zero charge)
template <typename AT>
__device__ __forceinline__ void load_point(const SymArgs &a, int64_t p, int lane, double &x, double &y,
                                           double &z, AT &ur, AT &ui) {
    using C2 = typename c2_of<AT>::type;
    if (p < a.ng) {
        x = a.px[p];
        y = a.py[p];
        z = a.pz[p];
        const C2 u = static_cast<const C2 *>(a.q)[p];
        ur = u.x;
        ui = u.y;
    } else {
        x = a.far[0] + a.far_step * lane;
        y = a.far[1];
        z = a.far[2];
        ur = 0;
        ui = 0;
    }
}

template <typename AT>
__device__ __forceinline__ void pair_e(double dx, double dy, double dz, const SymArgs &a, AT kk, AT &er, AT &ei) {
    AT ir2, kr;
    if constexpr (sizeof(AT) == 4) geom_f32<false>(dx, dy, dz, kk, a.kphase, er, ei, ir2, kr);
    else geom_f64<false>(dx, dy, dz, a.k, a.kphase, er, ei, ir2, kr);
}

// e = exp(i k r)/r and F = e (i k r - 1)/r^2 of one pair
template <typename AT>
__device__ __forceinline__ void pair_ef(double dx, double dy, double dz, const SymArgs &a, AT kk, AT &er, AT &ei,
                                        AT &fr, AT &fi) {
    AT ir2, kr;
    if constexpr (sizeof(AT) == 4) geom_f32<false>(dx, dy, dz, kk, a.kphase, er, ei, ir2, kr);
    else geom_f64<false>(dx, dy, dz, a.k, a.kphase, er, ei, ir2, kr);
    fr = ir2 * fma(-ei, kr, -er);
    fi = ir2 * fma(er, kr, -ei);
}

// v' and value of point p of a tile (padding lanes: zero)
template <typename AT>
__device__ __forceinline__ void load_t(const double *__restrict__ vx, const double *__restrict__ vy,
                                       const double *__restrict__ vz, const double2 *__restrict__ xv, int64_t p,
                                       int64_t count, AT &v0, AT &v1, AT &v2, AT &wr, AT &wi) {
    if (p < count) {
        v0 = static_cast<AT>(vx[p]);
        v1 = static_cast<AT>(vy[p]);
        v2 = static_cast<AT>(vz[p]);
        const double2 w = xv[p];
        wr = static_cast<AT>(w.x);
        wi = static_cast<AT>(w.y);
    } else {
        v0 = v1 = v2 = wr = wi = 0;
    }
}

// d . v' with d the FP64 difference: in FP32 from d rounded once on the FP32
// path (the product feeds an amplitude, not a phase), in FP64 otherwise
template <typename AT>
__device__ __forceinline__ AT dot_v(AT dxa, AT dya, AT dza, AT v0, AT v1, AT v2) {
    return fma(dxa, v0, fma(dya, v1, dza * v2));
}

// One slot partial, the FP64 sum over a partner group: FP32 kernels store it
// rounded to float2 (half the bytes written and read back by the reduction),
// FP64 kernels as double2.
template <typename AT>
__device__ __forceinline__ void store_slot(void *base, int64_t i, double re, double im) {
    if constexpr (sizeof(AT) == 4)
        static_cast<float2 *>(base)[i] = make_float2(static_cast<float>(re), static_cast<float>(im));
    else
        static_cast<double2 *>(base)[i] = make_double2(re, im);
}

// Waves per SIMD the compiler must leave room for, where that costs no
// instruction in the pair loop: the FP64 single-layer variant with groups of
// 8 (one-column products of the largest meshes) and the FP32 forward
// grad-alpha variants (6 waves, which their LDS tile allows too).
constexpr int sym_min_waves(int g, bool f64, bool t, bool adj) {
    return (g == 8 && f64 && !t) ? 4 : ((t && !adj && !f64) ? 6 : 1);
}

template <int G, typename AT, bool T, bool ADJ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sym_min_waves(G, sizeof(AT) == 8, T, ADJ))))
void sym_kernel(SymArgs a) {
    static_assert(T || !ADJ, "the adjoint variant of the symmetric kernel is the grad-alpha one");
    using C2 = typename c2_of<AT>::type;
    // per-wave copies of the B tile, stored twice in a row (entries 0..127) so
    // that step st reads entry lane + 64 - st without wrapping; one block per
    // wave, so the arrays sit at fixed offsets from one address
    struct BTileS {
        double x[128], y[128], z[128];
        C2 u[128];
    };
    struct BTileT {
        double x[128], y[128], z[128];
        C2 u[128];
        AT vx[128], vy[128], vz[128];
        C2 w[128];
    };
    struct BTileA {
        double x[128], y[128], z[128];
        C2 u[128];
        AT vx[128], vy[128], vz[128];
        C2 w[128];
        AT s[128];  // -s' of the B points
    };
    using BTile = typename std::conditional<ADJ, BTileA, typename std::conditional<T, BTileT, BTileS>::type>::type;
    __shared__ BTile lb[kWavesPerBlock];
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int xcd = blockIdx.x % kXcds;
    const int64_t waves_x = static_cast<int64_t>(gridDim.x / kXcds) * kWavesPerBlock;
    const int64_t w = static_cast<int64_t>(blockIdx.x / kXcds) * kWavesPerBlock + wib;
    const int64_t lo = a.xr[xcd], hi = a.xr[xcd + 1];
    const AT kk = static_cast<AT>(a.k);
    BTile &B = lb[wib];

    for (int64_t it = lo + w; it < hi; it += waves_x) {
        // item -> (I, J), I <= J, row by row: row I holds groups - I items and
        // starts at S(I) = I (2 groups - I + 1) / 2; I is the root of S(I) = it,
        // rounded down, then corrected in integers
        const int64_t g2 = 2 * static_cast<int64_t>(a.groups) + 1;
        int64_t r = static_cast<int64_t>((static_cast<double>(g2) - sqrt(static_cast<double>(g2 * g2 - 8 * it))) * 0.5);
        r = r < 0 ? 0 : (r >= a.groups ? a.groups - 1 : r);
        while (r > 0 && r * (g2 - r) / 2 > it) --r;
        while (r + 1 < a.groups && (r + 1) * (g2 - r - 1) / 2 <= it) ++r;
        const int I = static_cast<int>(r);
        const int J = static_cast<int>(r + (it - r * (g2 - r) / 2));
        // whether any tile of either group holds a cell with v' != 0 (wave-uniform)
        bool item_t = false;
        if constexpr (T) {
            for (int t = 0; t < G; ++t) {
                const int ti = I * G + t, tj = J * G + t;
                if (ti < a.tiles && a.tile_t[ti]) item_t = true;
                if (tj < a.tiles && a.tile_t[tj]) item_t = true;
            }
        }

        // B-side sums per tile of group J; the A side of tile ta is complete
        // when its row of tile pairs ends (on the diagonal, I = J, its B-side
        // sum from the rows before is complete by then too) and is stored there
        double accBr[G], accBi[G];
#pragma unroll
        for (int t = 0; t < G; ++t) accBr[t] = accBi[t] = 0.0;

        for (int ta = 0; ta < G; ++ta) {
            const int at = I * G + ta;
            if (at >= a.tiles) break;
            double accAr = 0.0, accAi = 0.0;
            double xa, ya, za;
            AT uar, uai;
            load_point<AT>(a, static_cast<int64_t>(at) * 64 + lane, lane, xa, ya, za, uar, uai);
            AT va0 = 0, va1 = 0, va2 = 0, war = 0, wai = 0;
            if constexpr (T) {
                if (item_t) load_t<AT>(a.vx, a.vy, a.vz, a.xv, static_cast<int64_t>(at) * 64 + lane, a.ng, va0, va1, va2, war, wai);
            }
            AT sa = 0;
            if constexpr (ADJ) {
                const int64_t pa = static_cast<int64_t>(at) * 64 + lane;
                sa = pa < a.ng ? -static_cast<AT>(a.sw[pa]) : AT(0);
            }
            for (int tb = (I == J) ? ta : 0; tb < G; ++tb) {
                const int bt = J * G + tb;
                if (bt >= a.tiles) break;
                {
                    double xb, yb, zb;
                    AT ubr, ubi;
                    load_point<AT>(a, static_cast<int64_t>(bt) * 64 + lane, lane, xb, yb, zb, ubr, ubi);
                    C2 u;
                    u.x = ubr;
                    u.y = ubi;
                    B.x[lane] = B.x[lane + 64] = xb;
                    B.y[lane] = B.y[lane + 64] = yb;
                    B.z[lane] = B.z[lane + 64] = zb;
                    B.u[lane] = B.u[lane + 64] = u;
                    if constexpr (T) {
                        if (item_t) {
                            AT v0, v1, v2, wr, wi;
                            load_t<AT>(a.vx, a.vy, a.vz, a.xv, static_cast<int64_t>(bt) * 64 + lane, a.ng, v0, v1, v2, wr, wi);
                            C2 w;
                            w.x = wr;
                            w.y = wi;
                            B.vx[lane] = B.vx[lane + 64] = v0;
                            B.vy[lane] = B.vy[lane + 64] = v1;
                            B.vz[lane] = B.vz[lane + 64] = v2;
                            B.w[lane] = B.w[lane + 64] = w;
                        }
                        if constexpr (ADJ) {
                            const int64_t pb = static_cast<int64_t>(bt) * 64 + lane;
                            B.s[lane] = B.s[lane + 64] = pb < a.ng ? -static_cast<AT>(a.sw[pb]) : AT(0);
                        }
                    }
                }
                AT sAr = 0, sAi = 0, sBr = 0, sBi = 0;
                bool done = false;
                if constexpr (ADJ) {
                    if (item_t) {
                        // weights on the target side, charges mu
                        if (at == bt) {
                            for (int st = 1; st < 64; ++st) {
                                const int j = lane + 64 - st;
                                const double dx = xa - B.x[j], dy = ya - B.y[j], dz = za - B.z[j];
                                AT er, ei, fr, fi;
                                pair_ef<AT>(dx, dy, dz, a, kk, er, ei, fr, fi);
                                const AT qa = dot_v<AT>(static_cast<AT>(dx), static_cast<AT>(dy), static_cast<AT>(dz),
                                                        va0, va1, va2);
                                const AT car = fma(sa, er, -qa * fr), cai = fma(sa, ei, -qa * fi);
                                const C2 u = B.u[j];
                                sAr = fma(car, u.x, fma(-cai, u.y, sAr));
                                sAi = fma(car, u.y, fma(cai, u.x, sAi));
                            }
                        } else {
                            for (int st = 0; st < 64; ++st) {
                                const int j = lane + 64 - st;
                                const double dx = xa - B.x[j], dy = ya - B.y[j], dz = za - B.z[j];
                                AT er, ei, fr, fi;
                                pair_ef<AT>(dx, dy, dz, a, kk, er, ei, fr, fi);
                                const AT dxa = static_cast<AT>(dx), dya = static_cast<AT>(dy), dza = static_cast<AT>(dz);
                                // target a: (-s'_a e - F d.v'_a) mu_b
                                const AT qa = dot_v<AT>(dxa, dya, dza, va0, va1, va2);
                                const AT car = fma(sa, er, -qa * fr), cai = fma(sa, ei, -qa * fi);
                                const C2 u = B.u[j];
                                sAr = fma(car, u.x, fma(-cai, u.y, sAr));
                                sAi = fma(car, u.y, fma(cai, u.x, sAi));
                                // target b: (-s'_b e + F d.v'_b) mu_a
                                const AT qb = dot_v<AT>(dxa, dya, dza, B.vx[j], B.vy[j], B.vz[j]);
                                const AT sb = B.s[j];
                                const AT cbr = fma(sb, er, qb * fr), cbi = fma(sb, ei, qb * fi);
                                sBr = rot1(fma(cbr, uar, fma(-cbi, uai, sBr)));
                                sBi = rot1(fma(cbr, uai, fma(cbi, uar, sBi)));
                            }
                        }
                        done = true;
                    }
                } else if constexpr (T) {
                    if (item_t) {
                        // single layer and adjoint double layer together
                        if (at == bt) {
                            // the tile with itself: the 63 other points, target side only
                            for (int st = 1; st < 64; ++st) {
                                const int j = lane + 64 - st;
                                const double dx = xa - B.x[j], dy = ya - B.y[j], dz = za - B.z[j];
                                AT er, ei, fr, fi;
                                pair_ef<AT>(dx, dy, dz, a, kk, er, ei, fr, fi);
                                const C2 u = B.u[j], w = B.w[j];
                                const AT qb = dot_v<AT>(static_cast<AT>(dx), static_cast<AT>(dy), static_cast<AT>(dz),
                                                        B.vx[j], B.vy[j], B.vz[j]);
                                const AT tbr = qb * w.x, tbi = qb * w.y;
                                sAr = fma(er, u.x, fma(-ei, u.y, fma(fr, tbr, fma(-fi, tbi, sAr))));
                                sAi = fma(er, u.y, fma(ei, u.x, fma(fr, tbi, fma(fi, tbr, sAi))));
                            }
                        } else {
                            for (int st = 0; st < 64; ++st) {
                                const int j = lane + 64 - st;
                                const double dx = xa - B.x[j], dy = ya - B.y[j], dz = za - B.z[j];
                                AT er, ei, fr, fi;
                                pair_ef<AT>(dx, dy, dz, a, kk, er, ei, fr, fi);
                                const AT dxa = static_cast<AT>(dx), dya = static_cast<AT>(dy), dza = static_cast<AT>(dz);
                                const C2 u = B.u[j], w = B.w[j];
                                // target a: e u_b + F (d.v'_b) x_b
                                const AT qb = dot_v<AT>(dxa, dya, dza, B.vx[j], B.vy[j], B.vz[j]);
                                const AT tbr = qb * w.x, tbi = qb * w.y;
                                sAr = fma(er, u.x, fma(-ei, u.y, fma(fr, tbr, fma(-fi, tbi, sAr))));
                                sAi = fma(er, u.y, fma(ei, u.x, fma(fr, tbi, fma(fi, tbr, sAi))));
                                // target b: e u_a + F (-d.v'_a) x_a
                                const AT qa = -dot_v<AT>(dxa, dya, dza, va0, va1, va2);
                                const AT tar = qa * war, tai = qa * wai;
                                sBr = rot1(fma(er, uar, fma(-ei, uai, fma(fr, tar, fma(-fi, tai, sBr)))));
                                sBi = rot1(fma(er, uai, fma(ei, uar, fma(fr, tai, fma(fi, tar, sBi)))));
                            }
                        }
                        done = true;
                    }
                }
                if (done) {
                    // the adjoint double layer loop above covered this tile pair
                } else if (at == bt) {
                    // the tile with itself: the 63 other points, target side only
                    for (int st = 1; st < 64; ++st) {
                        const int j = lane + 64 - st;
                        AT er, ei;
                        pair_e<AT>(xa - B.x[j], ya - B.y[j], za - B.z[j], a, kk, er, ei);
                        const C2 u = B.u[j];
                        sAr = fma(er, u.x, fma(-ei, u.y, sAr));
                        sAi = fma(er, u.y, fma(ei, u.x, sAi));
                    }
                } else {
                    for (int st = 0; st < 64; ++st) {
                        // B point (lane - st) mod 64; its accumulator has moved st lanes up
                        const int j = lane + 64 - st;
                        AT er, ei;
                        pair_e<AT>(xa - B.x[j], ya - B.y[j], za - B.z[j], a, kk, er, ei);
                        const C2 u = B.u[j];
                        sAr = fma(er, u.x, fma(-ei, u.y, sAr));
                        sAi = fma(er, u.y, fma(ei, u.x, sAi));
                        sBr = rot1(fma(er, uar, fma(-ei, uai, sBr)));
                        sBi = rot1(fma(er, uai, fma(ei, uar, sBi)));
                    }
                    // 64 rotations: every B point's sum is back in its home lane
                }
                if constexpr (ADJ) {
                    if (!item_t) {
                        // single layer alone: the targets' weights after the sums
                        sAr *= sa;
                        sAi *= sa;
                        const AT sbh = B.s[lane];
                        sBr *= sbh;
                        sBi *= sbh;
                    }
                }
                accAr += static_cast<double>(sAr);
                accAi += static_cast<double>(sAi);
                // tile-indexed accumulators with compile-time register indices
#pragma unroll
                for (int t = 0; t < G; ++t) {
                    if (t == tb) {
                        accBr[t] += static_cast<double>(sBr);
                        accBi[t] += static_cast<double>(sBi);
                    }
                }
            }
            // group I receives slot J (on the diagonal with its B-side sums)
            const int64_t pa = static_cast<int64_t>(at) * 64 + lane;
            if (pa < a.ng) {
                if (I == J) {
#pragma unroll
                    for (int t = 0; t < G; ++t) {
                        if (t == ta) {
                            accAr += accBr[t];
                            accAi += accBi[t];
                        }
                    }
                }
                store_slot<AT>(a.part, static_cast<int64_t>(J) * a.ldp + pa, accAr, accAi);
            }
        }
        // group J receives slot I
        if (I != J) {
#pragma unroll
            for (int t = 0; t < G; ++t) {
                const int bt = J * G + t;
                const int64_t pb = static_cast<int64_t>(bt) * 64 + lane;
                if (bt < a.tiles && pb < a.ng) store_slot<AT>(a.part, static_cast<int64_t>(I) * a.ldp + pb, accBr[t], accBi[t]);
            }
        }
    }
}

// The partial sums a point receives, as one list of slots from two arrays:
// slot t < na is a[t * lda + offa + p], slot na + t is b[t * ldb + offb + p]
// (p: index of the point within its class, cells or faces); a32 / b32: the
// array holds float2 partials, else double2.
struct SlotList {
    const void *a;
    int na;
    int64_t lda, offa;
    const void *b;
    int nb;
    int64_t ldb, offb;
    bool a32 = false, b32 = false;
};

// sr + i si += slots t0 .. t1-1 of one array, added in slot order in FP64
template <typename P>
__device__ __forceinline__ void add_slots(const void *base, int64_t ld, int64_t off, int t0, int t1, double &sr,
                                          double &si) {
    const P *__restrict__ v = static_cast<const P *>(base) + off;
#pragma unroll 8
    for (int t = t0; t < t1; ++t) {
        const P e = v[static_cast<int64_t>(t) * ld];
        sr += static_cast<double>(e.x);
        si += static_cast<double>(e.y);
    }
}

// y = diag x + the sum of each point's slots.  A workgroup takes 64 points of
// one class (cells: workgroups 0 .. cell_blocks-1, then faces); wave w adds
// the w-th quarter of the slots, and the four quarter sums are added in wave
// order, so the order of the additions is fixed.  Four waves per 64 points
// keep enough loads in flight to stream the partials at HBM speed.
// The adjoint variant writes y = conj(diag) x + conj(w sum) with w = -s'_i
// (sp) for cells and 1 for faces.
template <bool ADJ>
__global__ __launch_bounds__(kBlock) void slot_reduce_kernel(int64_t n, int64_t nc, int64_t cell_blocks,
                                                             SlotList cells, SlotList faces,
                                                             const double2 *__restrict__ diag,
                                                             const double2 *__restrict__ x, double2 *__restrict__ y,
                                                             const double *__restrict__ sp) {
    __shared__ double2 red[kWavesPerBlock][64];
    const int lane = threadIdx.x & 63;
    const int w = static_cast<int>(threadIdx.x) >> 6;
    const bool cell = blockIdx.x < cell_blocks;
    const int64_t p = (cell ? static_cast<int64_t>(blockIdx.x) : static_cast<int64_t>(blockIdx.x) - cell_blocks) * 64 + lane;
    const int64_t count = cell ? nc : n - nc;
    const SlotList &L = cell ? cells : faces;
    const int total = L.na + L.nb;
    const int t0 = static_cast<int>(static_cast<int64_t>(total) * w / kWavesPerBlock);
    const int t1 = static_cast<int>(static_cast<int64_t>(total) * (w + 1) / kWavesPerBlock);
    double sr = 0.0, si = 0.0;
    if (p < count) {
        const int ea = t1 < L.na ? t1 : L.na;
        if (L.a32) add_slots<float2>(L.a, L.lda, L.offa + p, t0, ea, sr, si);
        else add_slots<double2>(L.a, L.lda, L.offa + p, t0, ea, sr, si);
        const int b0 = (t0 > L.na ? t0 : L.na) - L.na, b1 = t1 - L.na;
        if (L.b32) add_slots<float2>(L.b, L.ldb, L.offb + p, b0, b1, sr, si);
        else add_slots<double2>(L.b, L.ldb, L.offb + p, b0, b1, sr, si);
    }
    red[w][lane] = make_double2(sr, si);
    __syncthreads();
    if (w == 0 && p < count) {
        for (int q = 1; q < kWavesPerBlock; ++q) {
            sr += red[q][lane].x;
            si += red[q][lane].y;
        }
        const int64_t i = cell ? p : nc + p;
        const double2 d = diag[i], xv = x[i];
        if constexpr (ADJ) {
            const double w = (cell && sp) ? -sp[i] : 1.0;
            y[i] = make_double2(d.x * xv.x + d.y * xv.y + w * sr, d.x * xv.y - d.y * xv.x - w * si);
        } else {
            y[i] = make_double2(d.x * xv.x - d.y * xv.y + sr, d.x * xv.y + d.y * xv.x + si);
        }
    }
}

// ---------------------------------------------------------------------------
// Cell-face pairs, one evaluation per pair (one right-hand side): the single
// layer of cell c at face target f and the double layer (T and K terms) of
// face f at cell target c share the pair's distance, phase, sine and cosine:
//   y_f += e u_c,                 u_c = -s'_c x_c
//   y_c += e (i k r - 1) q x_f,   q = (x_c - y_f).v'_f / r^2
// and, with cells that carry grad alpha (T variant, items whose cell group
// holds one), the cell's adjoint double layer at the face:
//   y_f += e (i k r - 1) q' x_c,  q' = (y_f - x_c).v'_c / r^2
// The adjoint variant (charges mu = conj(lambda)) sums the transposed terms
// of the same pairs: the single layer at the cell with the face's charge
// (scaled by the cell's -s' afterwards) and the face's double layer with the
// cell's charge:
//   z_c += e mu_f,                z_f += e (i k r - 1) q mu_c
// With grad-alpha cells the cell's weights enter in the kernel:
//   z_c += (-s'_c e + e (i k r - 1) (y_f - x_c).v'_c / r^2) mu_f
// Lanes hold cells (tile A); the face tile B (positions, v', values) sits in
// the wave's LDS slice and the faces' single-layer sums rotate by DPP, as in
// sym_kernel.  Work items are (cell group I, face group J), every pair of
// groups.  Cells receive one partial per face group (slot J), faces one per
// cell group (slot I).
struct CfArgs {
    int64_t nc, nf;                  // cells (points 0 .. nc-1), faces (points nc .. nc+nf-1)
    const double *__restrict__ px;
    const double *__restrict__ py;
    const double *__restrict__ pz;
    const double *__restrict__ vx;   // v' of the faces (nf entries, zero where a face has no weight)
    const double *__restrict__ vy;
    const double *__restrict__ vz;
    const void *__restrict__ qc;     // single-layer charges of the cells, complex AT
    const double2 *__restrict__ xf;  // values of the faces
    const void *__restrict__ qfa;    // adjoint: charges conj(lambda) of the faces, complex AT
    const double *__restrict__ sw;   // adjoint with grad-alpha cells: s' of the cells (weights in the kernel)
    // T variant: v' of the cells, their values, and per 64-cell tile whether any v' is nonzero
    const double *__restrict__ cvx;
    const double *__restrict__ cvy;
    const double *__restrict__ cvz;
    const double2 *__restrict__ xc;
    const int32_t *__restrict__ ctile_t;
    double k;
    double kphase;
    double far[3];
    double far_step;
    int ctiles, ftiles;
    int cgroups, fgroups;
    int64_t items;
    int64_t xr[kXcds + 1];           // item range of XCD x: [xr[x], xr[x + 1])
    void *__restrict__ pc;           // pc[slot * ldc + c], slot = face group (float2 or double2 as part)
    int64_t ldc;
    void *__restrict__ pf;           // pf[slot * ldf + f], slot = cell group
    int64_t ldf;
};

template <int G, typename AT, bool T, bool ADJ>
__global__ __launch_bounds__(kBlock) void cf_kernel(CfArgs a) {

    using C2 = typename c2_of<AT>::type;
    struct FTile {
        double x[128], y[128], z[128], vx[128], vy[128], vz[128];
        C2 u[128];
    };
    __shared__ FTile lb[kWavesPerBlock];
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int xcd = blockIdx.x % kXcds;
    const int64_t waves_x = static_cast<int64_t>(gridDim.x / kXcds) * kWavesPerBlock;
    const int64_t w = static_cast<int64_t>(blockIdx.x / kXcds) * kWavesPerBlock + wib;
    const int64_t lo = a.xr[xcd], hi = a.xr[xcd + 1];
    const AT kk = static_cast<AT>(a.k);
    FTile &B = lb[wib];

    for (int64_t it = lo + w; it < hi; it += waves_x) {
        const int I = static_cast<int>(it / a.fgroups);
        const int J = static_cast<int>(it - static_cast<int64_t>(I) * a.fgroups);
        bool item_t = false;
        if constexpr (T) {
            for (int t = 0; t < G; ++t) {
                const int ti = I * G + t;
                if (ti < a.ctiles && a.ctile_t[ti]) item_t = true;
            }
        }
        // the faces' sums per tile of group J; a cell tile's sum is complete
        // when its row of tile pairs ends and is stored there
        double accBr[G], accBi[G];
#pragma unroll
        for (int t = 0; t < G; ++t) accBr[t] = accBi[t] = 0.0;

        for (int ta = 0; ta < G; ++ta) {
            const int at = I * G + ta;
            if (at >= a.ctiles) break;
            const int64_t c = static_cast<int64_t>(at) * 64 + lane;
            double accAr = 0.0, accAi = 0.0;
            double xa, ya, za;
            AT uar, uai;
            if (c < a.nc) {
                xa = a.px[c];
                ya = a.py[c];
                za = a.pz[c];
                const C2 u = static_cast<const C2 *>(a.qc)[c];
                uar = u.x;
                uai = u.y;
            } else {
                xa = a.far[0] + a.far_step * lane;
                ya = a.far[1];
                za = a.far[2];
                uar = uai = 0;
            }
            double va0 = 0, va1 = 0, va2 = 0;
            AT war = 0, wai = 0;
            AT sa = 0;
            if constexpr (T && ADJ) {
                if (c < a.nc) sa = -static_cast<AT>(a.sw[c]);
            }
            if constexpr (T) {
                if (item_t && c < a.nc) {
                    va0 = a.cvx[c];
                    va1 = a.cvy[c];
                    va2 = a.cvz[c];
                    const double2 w = a.xc[c];
                    war = static_cast<AT>(w.x);
                    wai = static_cast<AT>(w.y);
                }
            }
            for (int tb = 0; tb < G; ++tb) {
                const int bt = J * G + tb;
                if (bt >= a.ftiles) break;
                {
                    const int64_t f = static_cast<int64_t>(bt) * 64 + lane;
                    double xb, yb, zb, wx = 0, wy = 0, wz = 0;
                    C2 u;
                    if (f < a.nf) {
                        xb = a.px[a.nc + f];
                        yb = a.py[a.nc + f];
                        zb = a.pz[a.nc + f];
                        wx = a.vx[f];
                        wy = a.vy[f];
                        wz = a.vz[f];
                        if constexpr (ADJ) {
                            u = static_cast<const C2 *>(a.qfa)[f];
                        } else {
                            const double2 xv = a.xf[f];
                            u.x = static_cast<AT>(xv.x);
                            u.y = static_cast<AT>(xv.y);
                        }
                    } else {
                        // padding faces: far points apart from the padding cells, v' = 0, value 0
                        xb = a.far[0] + a.far_step * (lane + 64);
                        yb = a.far[1];
                        zb = a.far[2];
                        u.x = 0;
                        u.y = 0;
                    }
                    B.x[lane] = B.x[lane + 64] = xb;
                    B.y[lane] = B.y[lane + 64] = yb;
                    B.z[lane] = B.z[lane + 64] = zb;
                    B.vx[lane] = B.vx[lane + 64] = wx;
                    B.vy[lane] = B.vy[lane + 64] = wy;
                    B.vz[lane] = B.vz[lane + 64] = wz;
                    B.u[lane] = B.u[lane + 64] = u;
                }
                AT sAr = 0, sAi = 0, sBr = 0, sBi = 0;
                bool done = false;
                if constexpr (T && ADJ) {
                    if (item_t) {
                        for (int st = 0; st < 64; ++st) {
                            const int j = lane + 64 - st;
                            const double dx = xa - B.x[j], dy = ya - B.y[j], dz = za - B.z[j];
                            AT er, ei, ir2, kr;
                            if constexpr (sizeof(AT) == 4) geom_f32<false>(dx, dy, dz, kk, a.kphase, er, ei, ir2, kr);
                            else geom_f64<false>(dx, dy, dz, a.k, a.kphase, er, ei, ir2, kr);
                            const AT fr = ir2 * fma(-ei, kr, -er);
                            const AT fi = ir2 * fma(er, kr, -ei);
                            // cell target: (-s'_c e - F d.v'_c) mu_f
                            const AT qa = static_cast<AT>(fma(dx, va0, fma(dy, va1, dz * va2)));
                            const AT car = fma(sa, er, -qa * fr), cai = fma(sa, ei, -qa * fi);
                            const C2 u = B.u[j];
                            sAr = fma(car, u.x, fma(-cai, u.y, sAr));
                            sAi = fma(car, u.y, fma(cai, u.x, sAi));
                            // face target: F (d.v'_f) mu_c
                            const AT qq = static_cast<AT>(fma(dx, B.vx[j], fma(dy, B.vy[j], dz * B.vz[j])));
                            const AT cr = qq * fr, ci = qq * fi;
                            sBr = rot1(fma(cr, uar, fma(-ci, uai, sBr)));
                            sBi = rot1(fma(cr, uai, fma(ci, uar, sBi)));
                        }
                        done = true;
                    }
                } else if constexpr (T) {
                    if (item_t) {
                        for (int st = 0; st < 64; ++st) {
                            const int j = lane + 64 - st;
                            const double dx = xa - B.x[j], dy = ya - B.y[j], dz = za - B.z[j];
                            AT er, ei, ir2, kr;
                            if constexpr (sizeof(AT) == 4) geom_f32<false>(dx, dy, dz, kk, a.kphase, er, ei, ir2, kr);
                            else geom_f64<false>(dx, dy, dz, a.k, a.kphase, er, ei, ir2, kr);
                            // F = e (i k r - 1) / r^2
                            const AT fr = ir2 * fma(-ei, kr, -er);
                            const AT fi = ir2 * fma(er, kr, -ei);
                            // double layer of the face at the cell
                            const AT qq = static_cast<AT>(fma(dx, B.vx[j], fma(dy, B.vy[j], dz * B.vz[j])));
                            const C2 u = B.u[j];
                            const AT tr = qq * u.x, ti = qq * u.y;
                            sAr = fma(fr, tr, fma(-fi, ti, sAr));
                            sAi = fma(fr, ti, fma(fi, tr, sAi));
                            // single layer and adjoint double layer of the cell at the face
                            const AT qc = -static_cast<AT>(fma(dx, va0, fma(dy, va1, dz * va2)));
                            const AT cr = qc * war, ci = qc * wai;
                            sBr = rot1(fma(er, uar, fma(-ei, uai, fma(fr, cr, fma(-fi, ci, sBr)))));
                            sBi = rot1(fma(er, uai, fma(ei, uar, fma(fr, ci, fma(fi, cr, sBi)))));
                        }
                        done = true;
                    }
                }
                if constexpr (ADJ) {
                    for (int st = 0; st < (done ? 0 : 64); ++st) {
                        const int j = lane + 64 - st;
                        const double dx = xa - B.x[j], dy = ya - B.y[j], dz = za - B.z[j];
                        AT er, ei, ir2, kr;
                        if constexpr (sizeof(AT) == 4) geom_f32<false>(dx, dy, dz, kk, a.kphase, er, ei, ir2, kr);
                        else geom_f64<false>(dx, dy, dz, a.k, a.kphase, er, ei, ir2, kr);
                        // single layer at the cell, with the face's charge
                        const C2 u = B.u[j];
                        sAr = fma(er, u.x, fma(-ei, u.y, sAr));
                        sAi = fma(er, u.y, fma(ei, u.x, sAi));
                        // the face's double layer, with the cell's charge
                        const AT qq = static_cast<AT>(fma(dx, B.vx[j], fma(dy, B.vy[j], dz * B.vz[j]))) * ir2;
                        const AT cr = qq * fma(-ei, kr, -er);
                        const AT ci = qq * fma(er, kr, -ei);
                        sBr = rot1(fma(cr, uar, fma(-ci, uai, sBr)));
                        sBi = rot1(fma(cr, uai, fma(ci, uar, sBi)));
                    }
                    if constexpr (T) {
                        // items without grad-alpha cells: the cells' weights after the sums
                        if (!done) {
                            sAr *= sa;
                            sAi *= sa;
                        }
                    }
                    done = true;
                }
                for (int st = 0; st < (done ? 0 : 64); ++st) {
                    // face (lane - st) mod 64; its single-layer sum has moved st lanes up
                    const int j = lane + 64 - st;
                    const double dx = xa - B.x[j], dy = ya - B.y[j], dz = za - B.z[j];
                    AT er, ei, ir2, kr;
                    if constexpr (sizeof(AT) == 4) geom_f32<false>(dx, dy, dz, kk, a.kphase, er, ei, ir2, kr);
                    else geom_f64<false>(dx, dy, dz, a.k, a.kphase, er, ei, ir2, kr);
                    // double layer of the face at the cell
                    const AT qq = static_cast<AT>(fma(dx, B.vx[j], fma(dy, B.vy[j], dz * B.vz[j]))) * ir2;
                    const AT cr = qq * fma(-ei, kr, -er);
                    const AT ci = qq * fma(er, kr, -ei);
                    const C2 u = B.u[j];
                    sAr = fma(cr, u.x, fma(-ci, u.y, sAr));
                    sAi = fma(cr, u.y, fma(ci, u.x, sAi));
                    // single layer of the cell at the face
                    sBr = rot1(fma(er, uar, fma(-ei, uai, sBr)));
                    sBi = rot1(fma(er, uai, fma(ei, uar, sBi)));
                }
                accAr += static_cast<double>(sAr);
                accAi += static_cast<double>(sAi);
#pragma unroll
                for (int t = 0; t < G; ++t) {
                    if (t == tb) {
                        accBr[t] += static_cast<double>(sBr);
                        accBi[t] += static_cast<double>(sBi);
                    }
                }
            }
            if (c < a.nc) store_slot<AT>(a.pc, static_cast<int64_t>(J) * a.ldc + c, accAr, accAi);
        }
#pragma unroll
        for (int t = 0; t < G; ++t) {
            const int bt = J * G + t;
            const int64_t f = static_cast<int64_t>(bt) * 64 + lane;
            if (bt < a.ftiles && f < a.nf) store_slot<AT>(a.pf, static_cast<int64_t>(I) * a.ldf + f, accBr[t], accBi[t]);
        }
    }
}

template <int G, typename AT>
const void *sym_ptr(bool t, bool adj) {
    if (adj) return reinterpret_cast<const void *>(&sym_kernel<G, AT, true, true>);
    return t ? reinterpret_cast<const void *>(&sym_kernel<G, AT, true, false>)
             : reinterpret_cast<const void *>(&sym_kernel<G, AT, false, false>);
}

const void *pick_sym(int g, bool f32, bool t, bool adj) {
    if (g == 1) return f32 ? sym_ptr<1, float>(t, adj) : sym_ptr<1, double>(t, adj);
    if (g == 2) return f32 ? sym_ptr<2, float>(t, adj) : sym_ptr<2, double>(t, adj);
    if (g == 4) return f32 ? sym_ptr<4, float>(t, adj) : sym_ptr<4, double>(t, adj);
    if (g == 8) return f32 ? sym_ptr<8, float>(t, adj) : sym_ptr<8, double>(t, adj);
    return nullptr;
}

void launch_slot_reduce(int64_t n, int64_t nc, const SlotList &cells, const SlotList &faces,
                        const double2 *diag, const double2 *x, double2 *y, hipStream_t s, bool adj = false,
                        const double *adj_sp = nullptr) {
    const int64_t cell_blocks = (nc + 63) / 64, face_blocks = (n - nc + 63) / 64;
    const int64_t blocks = cell_blocks + face_blocks;
    if (blocks > 0x7fffffff) fail(VSIE_E_INVALID, "slot reduction: too many points");
    if (adj)
        hipLaunchKernelGGL(slot_reduce_kernel<true>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, n, nc,
                           cell_blocks, cells, faces, diag, x, y, adj_sp);
    else
        hipLaunchKernelGGL(slot_reduce_kernel<false>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, n, nc,
                           cell_blocks, cells, faces, diag, x, y, adj_sp);
    VSIE_HIP(hipGetLastError());
}

}  // namespace

// Workgroups for one item per wave: 8 XCD ranges of at most ceil(items / 8)
// items, kWavesPerBlock waves per workgroup, workgroup b on range b mod 8.
int64_t one_item_per_wave_grid(int64_t items) {
    const int64_t per_xcd = (items + kXcds - 1) / kXcds;
    const int64_t grid = kXcds * std::max<int64_t>(1, (per_xcd + kWavesPerBlock - 1) / kWavesPerBlock);
    if (grid > 0x7fffffff) fail(VSIE_E_INVALID, "pair kernel: too many work items for one launch");
    return grid;
}

namespace {

// the same for ranges of unequal length: one wave per item of the longest range
int64_t ranges_grid(const int64_t *xr) {
    int64_t most = 1;
    for (int x = 0; x < kXcds; ++x) most = std::max<int64_t>(most, xr[x + 1] - xr[x]);
    const int64_t grid = kXcds * ((most + kWavesPerBlock - 1) / kWavesPerBlock);
    if (grid > 0x7fffffff) fail(VSIE_E_INVALID, "pair kernel: too many work items for one launch");
    return grid;
}

void equal_ranges(int64_t items, int64_t *xr) {
    for (int x = 0; x <= kXcds; ++x) xr[x] = items * x / kXcds;
}

// Boundaries of 8 contiguous item ranges of equal cost, items in order, with
// cost(it) = weight for flagged items and 1 otherwise; flagged(it) is called
// once per item in increasing order.
template <typename Flag>
void cost_ranges(int64_t items, double weight, Flag flagged, int64_t *xr) {
    std::vector<unsigned char> f(static_cast<size_t>(items));
    double total = 0.0;
    for (int64_t it = 0; it < items; ++it) {
        f[static_cast<size_t>(it)] = flagged(it) ? 1 : 0;
        total += f[static_cast<size_t>(it)] ? weight : 1.0;
    }
    xr[0] = 0;
    double acc = 0.0;
    int x = 1;
    for (int64_t it = 0; it < items && x < kXcds; ++it) {
        acc += f[static_cast<size_t>(it)] ? weight : 1.0;
        while (x < kXcds && acc >= total * x / kXcds) xr[x++] = it + 1;
    }
    while (x < kXcds) xr[x++] = items;
    xr[kXcds] = items;
}

}  // namespace

void sym_cost_ranges(int64_t ng, int g, const std::vector<int32_t> &tile_t, double weight, int64_t *xr) {
    const int64_t tiles = (ng + 63) / 64, groups = sym_slots(ng, g);
    const int64_t items = groups * (groups + 1) / 2;
    std::vector<char> gt(static_cast<size_t>(groups), 0);
    for (int64_t t = 0; t < tiles && t < static_cast<int64_t>(tile_t.size()); ++t)
        if (tile_t[static_cast<size_t>(t)]) gt[static_cast<size_t>(t / g)] = 1;
    // item order: row I, then J = I .. groups - 1
    int64_t I = 0, J = 0;
    cost_ranges(items, weight, [&](int64_t) {
        const bool r = gt[static_cast<size_t>(I)] || gt[static_cast<size_t>(J)];
        if (++J == groups) J = ++I;
        return r;
    }, xr);
}

void cf_cost_ranges(int64_t nc, int64_t nf, const std::vector<int32_t> &tile_t, double weight, int64_t *xr) {
    const int64_t ctiles = (nc + 63) / 64, cgroups = cf_groups(nc), fgroups = cf_groups(nf);
    std::vector<char> gt(static_cast<size_t>(cgroups), 0);
    for (int64_t t = 0; t < ctiles && t < static_cast<int64_t>(tile_t.size()); ++t)
        if (tile_t[static_cast<size_t>(t)]) gt[static_cast<size_t>(t / kCfGroup)] = 1;
    // item order: cell group I, then face group J
    cost_ranges(cgroups * fgroups, weight, [&](int64_t it) { return gt[static_cast<size_t>(it / fgroups)] != 0; }, xr);
}

bool sym_groups_ok(int g) { return g == 1 || g == 2 || g == 4 || g == 8; }

int64_t sym_slots(int64_t ng, int g) {
    const int64_t tiles = (ng + 63) / 64;
    return (tiles + g - 1) / g;
}

void launch_sym(const SymJob &J, hipStream_t s, PairProfiler *prof) {
    if (J.ng <= 0) return;
    if (!sym_groups_ok(J.g)) fail(VSIE_E_INVALID, "symmetric pair kernel: unsupported group size");
    const bool f32 = J.prec == VSIE_FP32;
    SymArgs a{};
    a.ng = J.ng;
    a.px = J.px;
    a.py = J.py;
    a.pz = J.pz;
    a.q = J.q;
    a.k = J.k;
    a.kphase = f32 ? J.k / kTwoPi : J.k / kPi;
    for (int d = 0; d < 3; ++d) a.far[d] = J.far[d];
    a.far_step = J.far_step;
    a.tiles = static_cast<int>((J.ng + 63) / 64);
    a.groups = static_cast<int>(sym_slots(J.ng, J.g));
    a.items = static_cast<int64_t>(a.groups) * (a.groups + 1) / 2;
    if (J.xr) {
        if (J.xr[0] != 0 || J.xr[kXcds] != a.items) fail(VSIE_E_INVALID, "symmetric pair kernel: item ranges do not cover the items");
        for (int x = 0; x < kXcds; ++x)
            if (J.xr[x] > J.xr[x + 1]) fail(VSIE_E_INVALID, "symmetric pair kernel: item ranges out of order");
        for (int x = 0; x <= kXcds; ++x) a.xr[x] = J.xr[x];
    } else {
        equal_ranges(a.items, a.xr);
    }
    a.part = J.part;
    a.ldp = J.ldp;
    a.vx = J.vx;
    a.vy = J.vy;
    a.vz = J.vz;
    a.xv = J.xv;
    a.tile_t = J.tile_t;
    a.sw = J.sw;
    if (J.ldp < J.ng) fail(VSIE_E_INVALID, "symmetric pair kernel: partial stride below the cell count");
    const bool t = J.vx != nullptr;
    if (t && !(J.vy && J.vz && J.xv && J.tile_t)) fail(VSIE_E_INVALID, "symmetric pair kernel: incomplete T data");
    if (J.adj && !(t && J.sw)) fail(VSIE_E_INVALID, "symmetric pair kernel: the adjoint variant needs the T data and s'");
    const void *kp = pick_sym(J.g, f32, t, J.adj);
    const int64_t grid = ranges_grid(a.xr);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (prof && prof->on) {
        ev0 = prof_take_event(prof);
        ev1 = prof_take_event(prof);
        VSIE_HIP(hipEventRecord(ev0, s));
    }
    hipLaunchKernelGGL(reinterpret_cast<void (*)(SymArgs)>(const_cast<void *>(kp)), dim3(static_cast<unsigned>(grid)),
                       dim3(kBlock), 0, s, a);
    VSIE_HIP(hipGetLastError());
    if (prof && prof->on) {
        VSIE_HIP(hipEventRecord(ev1, s));
        const double pairs = static_cast<double>(J.ng) * (J.ng - 1);
        prof->recs.push_back(PairProfiler::Rec{ev0, ev1, J.prof_kind + (f32 ? 1 : 0), pairs, pairs});
    }
}

// y = diag x + (cells: symmetric slots; faces: one-sided single-layer chunk
// partials) + the double-layer chunk partials (stride n, global index)
void launch_sym_reduce(int64_t n, int64_t n_vol, int n_slots, const void *sym, bool sym32, int64_t ldp,
                       int n_face_parts, const double2 *face, int n_f_parts, const double2 *fpart,
                       const double2 *diag, const double2 *x, double2 *y, hipStream_t s) {
    if (n == 0) return;
    const int64_t nf = n - n_vol;
    const SlotList cells{sym, n_slots, ldp, 0, fpart, n_f_parts, n, 0, sym32, false};
    const SlotList faces{face, n_face_parts, nf, 0, fpart, n_f_parts, n, n_vol};
    launch_slot_reduce(n, n_vol, cells, faces, diag, x, y, s);
}

int64_t cf_groups(int64_t count) { return ((count + 63) / 64 + kCfGroup - 1) / kCfGroup; }

void launch_cf(const CfJob &J, hipStream_t s, PairProfiler *prof) {
    if (J.nc <= 0 || J.nf <= 0) return;
    const bool f32 = J.prec == VSIE_FP32;
    CfArgs a{};
    a.nc = J.nc;
    a.nf = J.nf;
    a.px = J.px;
    a.py = J.py;
    a.pz = J.pz;
    a.vx = J.vx;
    a.vy = J.vy;
    a.vz = J.vz;
    a.qc = J.qc;
    a.xf = J.xf;
    a.qfa = J.qfa;
    a.sw = J.sw;
    a.cvx = J.cvx;
    a.cvy = J.cvy;
    a.cvz = J.cvz;
    a.xc = J.xc;
    a.ctile_t = J.ctile_t;
    a.k = J.k;
    a.kphase = f32 ? J.k / kTwoPi : J.k / kPi;
    for (int d = 0; d < 3; ++d) a.far[d] = J.far[d];
    a.far_step = J.far_step;
    a.ctiles = static_cast<int>((J.nc + 63) / 64);
    a.ftiles = static_cast<int>((J.nf + 63) / 64);
    a.cgroups = static_cast<int>(cf_groups(J.nc));
    a.fgroups = static_cast<int>(cf_groups(J.nf));
    a.items = static_cast<int64_t>(a.cgroups) * a.fgroups;
    if (J.xr) {
        if (J.xr[0] != 0 || J.xr[kXcds] != a.items) fail(VSIE_E_INVALID, "cell-face kernel: item ranges do not cover the items");
        for (int x = 0; x < kXcds; ++x)
            if (J.xr[x] > J.xr[x + 1]) fail(VSIE_E_INVALID, "cell-face kernel: item ranges out of order");
        for (int x = 0; x <= kXcds; ++x) a.xr[x] = J.xr[x];
    } else {
        equal_ranges(a.items, a.xr);
    }
    a.pc = J.pc;
    a.ldc = J.nc;
    a.pf = J.pf;
    a.ldf = J.nf;
    const bool t = J.cvx != nullptr;
    if (t && !(J.cvy && J.cvz && J.xc && J.ctile_t)) fail(VSIE_E_INVALID, "cell-face kernel: incomplete T data");
    if (t && J.adj && !J.sw) fail(VSIE_E_INVALID, "cell-face kernel: the adjoint with grad-alpha cells needs s'");
    if (!(J.adj ? J.qfa != nullptr : J.xf != nullptr) || !J.vx || !J.vy || !J.vz)
        fail(VSIE_E_INVALID, "cell-face kernel: missing face data");
    const void *kp = nullptr;
    if (J.adj && t) kp = f32 ? reinterpret_cast<const void *>(&cf_kernel<kCfGroup, float, true, true>)
                             : reinterpret_cast<const void *>(&cf_kernel<kCfGroup, double, true, true>);
    else if (J.adj) kp = f32 ? reinterpret_cast<const void *>(&cf_kernel<kCfGroup, float, false, true>)
                             : reinterpret_cast<const void *>(&cf_kernel<kCfGroup, double, false, true>);
    else if (t) kp = f32 ? reinterpret_cast<const void *>(&cf_kernel<kCfGroup, float, true, false>)
                         : reinterpret_cast<const void *>(&cf_kernel<kCfGroup, double, true, false>);
    else kp = f32 ? reinterpret_cast<const void *>(&cf_kernel<kCfGroup, float, false, false>)
                  : reinterpret_cast<const void *>(&cf_kernel<kCfGroup, double, false, false>);
    const int64_t grid = ranges_grid(a.xr);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (prof && prof->on) {
        ev0 = prof_take_event(prof);
        ev1 = prof_take_event(prof);
        VSIE_HIP(hipEventRecord(ev0, s));
    }
    hipLaunchKernelGGL(reinterpret_cast<void (*)(CfArgs)>(const_cast<void *>(kp)), dim3(static_cast<unsigned>(grid)),
                       dim3(kBlock), 0, s, a);
    VSIE_HIP(hipGetLastError());
    if (prof && prof->on) {
        VSIE_HIP(hipEventRecord(ev1, s));
        const double pairs = 2.0 * static_cast<double>(J.nc) * J.nf;
        prof->recs.push_back(PairProfiler::Rec{ev0, ev1, 12 + (f32 ? 1 : 0), pairs, pairs});
    }
}

// y = diag x + (cells: symmetric slots + cell-face slots; faces: cell-face
// slots + face-face chunk partials); one right-hand side
void launch_cf_reduce(int64_t n, int64_t nc, bool slots32, int n_sym, const void *sym, int n_cs, const void *pc,
                      int n_fs, const void *pf, int n_ff, const void *ff, bool ff32, const double2 *diag,
                      const double2 *x, double2 *y, hipStream_t s, bool adj, const double *adj_sp) {
    if (n == 0) return;
    const int64_t nf = n - nc;
    const SlotList cells{sym, n_sym, nc, 0, pc, n_cs, nc, 0, slots32, slots32};
    const SlotList faces{pf, n_fs, nf, 0, ff, n_ff, nf, 0, slots32, ff32};
    launch_slot_reduce(n, nc, cells, faces, diag, x, y, s, adj, adj_sp);
}

}  // namespace vsie
