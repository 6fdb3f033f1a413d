// O(n) kernels of the VSIE path: per-element weights, charge packing,
// reduction of pair-kernel partial sums with the diagonal, plane waves, and
// the dense complex vector operations of the Krylov solver.
#include "vsie_internal.h"

namespace vsie {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kInv4Pi = 1.0 / (4.0 * kPi);
constexpr int kT = 256;

inline unsigned blocks_for(int64_t n, int per = kT) {
    return static_cast<unsigned>((n + per - 1) / per);
}

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Integral of G_k(0, y) over the ball of radius a (the paper's equal-volume
// sphere self-term): ((1 - i k a) exp(i k a) - 1) / k^2, evaluated through its
// power series (1/k^2) sum_{n>=2} (i k a)^n (1 - n) / n! when k a < 0.5.
__device__ double2 ball_self_integral(double a, double k) {
    const double ka = k * a;
    if (ka < 0.5) {
        // term_n = (i k a)^n / n!, starting at n = 2
        double2 t = make_double2(-0.5 * ka * ka, 0.0);
        double2 acc = make_double2(-t.x, -t.y);  // (1 - 2) * term_2
        for (int n = 3; n < 30; ++n) {
            t = cmul(t, make_double2(0.0, ka / n));
            acc.x += (1 - n) * t.x;
            acc.y += (1 - n) * t.y;
        }
        return make_double2(acc.x / (k * k), acc.y / (k * k));
    }
    double sn, cs;
    sincos(ka, &sn, &cs);
    // (1 - i ka)(cs + i sn) - 1
    const double re = cs + ka * sn - 1.0;
    const double im = sn - ka * cs;
    return make_double2(re / (k * k), im / (k * k));
}

__global__ void weights_kernel(DeviceMesh m, const double *__restrict__ k0, int n_freq) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (e >= m.n) return;
    const double rho0 = m.rho0, c0 = m.c0;
    if (e < m.n_vol) {
        const double rho = m.vrho[e], c = m.vc[e], w = m.vw[e];
        const double contrast = rho0 / rho;              // 1 + alpha
        const double mass = contrast;                    // mass function inside a subdomain
        // grad alpha: explicit, or per-axis differences over same-subdomain neighbours
        double ga[3] = {0.0, 0.0, 0.0};
        if (m.vga) {
            for (int ax = 0; ax < 3; ++ax) ga[ax] = m.vga[3 * e + ax];
        } else if (m.vgr) {
            // alpha = rho0/rho - 1 (eq_alpha): grad alpha = -rho0 grad(rho) / rho^2
            for (int ax = 0; ax < 3; ++ax) ga[ax] = -rho0 * m.vgr[3 * e + ax] / (rho * rho);
        } else if (m.vnb) {
            const double *pc[3] = {m.px, m.py, m.pz};
            const int dom = m.vdom[e];
            for (int ax = 0; ax < 3; ++ax) {
                const int lo = m.vnb[6 * e + 2 * ax], hi = m.vnb[6 * e + 2 * ax + 1];
                const bool lok = lo >= 0 && m.vdom[lo] == dom;
                const bool hok = hi >= 0 && m.vdom[hi] == dom;
                if (!lok && !hok) continue;
                const int64_t a = lok ? lo : e, b = hok ? hi : e;
                const double aa = rho0 / m.vrho[a] - 1.0, ab = rho0 / m.vrho[b] - 1.0;
                ga[ax] = (ab - aa) / (pc[ax][b] - pc[ax][a]);
            }
        }
        m.vpx[e] = w * ga[0] * kInv4Pi;
        m.vpy[e] = w * ga[1] * kInv4Pi;
        m.vpz[e] = w * ga[2] * kInv4Pi;
        m.mass[e] = mass;
        const double a_eq = cbrt(3.0 * w / (4.0 * kPi));
        const double cr = c0 / c;
        for (int f = 0; f < n_freq; ++f) {
            const double k = k0[f];
            // |cell| (beta - k0^2 alpha) = |cell| (rho0/rho)(k_c^2 - k0^2), k_c = k0 c0 / c
            const double wt = contrast * k * k * (cr * cr - 1.0);
            m.sp[f * m.n + e] = w * wt * kInv4Pi;
            const double2 S = ball_self_integral(a_eq, k);
            m.diag[f * m.n + e] = make_double2(mass - wt * S.x, -wt * S.y);
        }
    } else {
        const int64_t q = e - m.n_vol;
        const double rin = m.vrho[m.scin[q]];
        const int co = m.scout[q];
        const double rout = co >= 0 ? m.vrho[co] : rho0;
        // alpha_inside - alpha_outside and the averaged contrast (mass function on Gamma)
        const double jump = rho0 / rin - rho0 / rout;
        const double mass = 0.5 * (rho0 / rin + rho0 / rout);
        const double g = -m.sarea[q] * jump * kInv4Pi;
        m.vpx[e] = g * m.snx[q];
        m.vpy[e] = g * m.sny[q];
        m.vpz[e] = g * m.snz[q];
        m.mass[e] = mass;
        for (int f = 0; f < n_freq; ++f) {
            m.sp[f * m.n + e] = 0.0;
            m.diag[f * m.n + e] = make_double2(mass, 0.0);
        }
    }
}

template <typename C2>
__device__ inline C2 to_c2(double re, double im);
template <> __device__ inline double2 to_c2<double2>(double re, double im) { return make_double2(re, im); }
template <> __device__ inline float2 to_c2<float2>(double re, double im) {
    return make_float2(static_cast<float>(re), static_cast<float>(im));
}

// charge[r * count + jj] = scale_jj * x[idx[jj] + r ldx] (conjugated first when conj_in),
// with scale_jj = -s'[idx[jj]] for the single-layer class, 1 otherwise.
template <typename C2>
__global__ void pack_kernel(int64_t count, const int32_t *__restrict__ idx,
                            const double *__restrict__ sp, int nrhs,
                            const double2 *__restrict__ x, int64_t ldx, bool conj_in,
                            C2 *__restrict__ out) {
    const int64_t jj = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (jj >= count) return;
    const int64_t j = idx ? idx[jj] : jj;
    const double sc = sp ? -sp[j] : 1.0;
    for (int r = 0; r < nrhs; ++r) {
        double2 v = x[j + r * ldx];
        if (conj_in) v.y = -v.y;
        out[jj + r * count] = to_c2<C2>(sc * v.x, sc * v.y);
    }
}

// Both source classes in one launch: threads 0 .. cg-1 pack the single-layer
// charges (as pack_kernel with sp), the next cf threads the double-layer ones.
template <typename C2>
__global__ void pack2_kernel(int64_t cg, const int32_t *__restrict__ idxg, const double *__restrict__ sp,
                             int64_t cf, const int32_t *__restrict__ idxf, int nrhs,
                             const double2 *__restrict__ x, int64_t ldx, bool conj_in, C2 *__restrict__ outg,
                             C2 *__restrict__ outf) {
    int64_t jj = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    const bool g = jj < cg;
    if (!g) jj -= cg;
    if (!g && jj >= cf) return;
    const int32_t *idx = g ? idxg : idxf;
    const int64_t count = g ? cg : cf;
    const int64_t j = idx ? idx[jj] : jj;
    const double sc = g ? -sp[j] : 1.0;
    C2 *out = g ? outg : outf;
    for (int r = 0; r < nrhs; ++r) {
        double2 v = x[j + r * ldx];
        if (conj_in) v.y = -v.y;
        out[jj + r * count] = to_c2<C2>(sc * v.x, sc * v.y);
    }
}

// y[i + r ldy] = d_i x[i + r ldx] + sum_c partial[(c nrhs + r) n_t + i],
// d_i = diag[i] (conjugated when conj_diag); diag == nullptr means d_i = 0.
__global__ void reduce_kernel(int64_t n_t, int nrhs, int n_parts, const double2 *__restrict__ part,
                              const double2 *__restrict__ diag, bool conj_diag,
                              const double2 *__restrict__ x, int64_t ldx, double2 *__restrict__ y,
                              int64_t ldy) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (i >= n_t) return;
    double2 d = diag ? diag[i] : make_double2(0.0, 0.0);
    if (conj_diag) d.y = -d.y;
    for (int r = 0; r < nrhs; ++r) {
        double2 acc = make_double2(0.0, 0.0);
        if (diag) acc = cmul(d, x[i + r * ldx]);
        for (int c = 0; c < n_parts; ++c) {
            const double2 p = part[(static_cast<int64_t>(c) * nrhs + r) * n_t + i];
            acc.x += p.x;
            acc.y += p.y;
        }
        y[i + r * ldy] = acc;
    }
}

// X2[i + r n] = Re x[i + r ldx], X2[i + (nrhs + r) n] = Im x[i + r ldx]  (FP32)
__global__ void pack_planar_kernel(int64_t n, int nrhs, const double2 *__restrict__ x, int64_t ldx,
                                   float *__restrict__ X2) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= n) return;
    const double2 v = x[i + r * ldx];
    X2[i + static_cast<int64_t>(r) * n] = static_cast<float>(v.x);
    X2[i + static_cast<int64_t>(nrhs + r) * n] = static_cast<float>(v.y);
}

// y = d x (conj(d) for the adjoint) + sum over slabs of the planar partials
// (see launch_reduce_planar), added in FP64
__global__ void reduce_planar_kernel(int64_t n, int nrhs, int n_parts, const float *__restrict__ part,
                                     const double2 *__restrict__ diag, bool adjoint,
                                     const double2 *__restrict__ x, int64_t ldx, double2 *__restrict__ y,
                                     int64_t ldy) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= n) return;
    double2 d = diag[i];
    if (adjoint) d.y = -d.y;
    double2 acc = cmul(d, x[i + r * ldx]);
    const int64_t blk = static_cast<int64_t>(2) * nrhs * n;  // one n x 2 nrhs product
    for (int c = 0; c < n_parts; ++c) {
        const float *P = part + 2 * c * blk, *Q = P + blk;
        const double pr = P[r * n + i], pi = P[(nrhs + r) * n + i];
        const double qr = Q[r * n + i], qi = Q[(nrhs + r) * n + i];
        if (!adjoint) {
            acc.x += pr - qi;
            acc.y += pi + qr;
        } else {
            acc.x += pr + qi;
            acc.y += pi - qr;
        }
    }
    y[i + r * ldy] = acc;
}

// y[idx[jj] + r ldy] += conj(scale_jj * sum_c partial[(c nrhs + r) count + jj]),
// scale_jj = -s'[idx[jj]] (single-layer class) or 1.
__global__ void scatter_conj_kernel(int64_t count, const int32_t *__restrict__ idx,
                                    const double *__restrict__ sp, int nrhs, int n_parts,
                                    const double2 *__restrict__ part, double2 *__restrict__ y,
                                    int64_t ldy) {
    const int64_t jj = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (jj >= count) return;
    const int64_t j = idx[jj];
    const double sc = sp ? -sp[j] : 1.0;
    for (int r = 0; r < nrhs; ++r) {
        double2 acc = make_double2(0.0, 0.0);
        for (int c = 0; c < n_parts; ++c) {
            const double2 p = part[(static_cast<int64_t>(c) * nrhs + r) * count + jj];
            acc.x += p.x;
            acc.y += p.y;
        }
        double2 v = y[j + r * ldy];
        v.x += sc * acc.x;
        v.y -= sc * acc.y;
        y[j + r * ldy] = v;
    }
}

// z[j + r ldz] = conj(sum_c P[c][4r][j]) / (4 pi),
// Z[j + (3r + a) ldZ] = conj(sum_c P[c][4r + 1 + a][j]) / (4 pi).
__global__ void sums_reduce_kernel(int64_t n, int nrhs, int n_parts, const double2 *__restrict__ part,
                                   double2 *__restrict__ z, int64_t ldz, double2 *__restrict__ Z,
                                   int64_t ldZ) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (j >= n) return;
    for (int r = 0; r < nrhs; ++r) {
        for (int comp = 0; comp < 4; ++comp) {
            double2 acc = make_double2(0.0, 0.0);
            for (int c = 0; c < n_parts; ++c) {
                const double2 p = part[(static_cast<int64_t>(c) * nrhs * 4 + 4 * r + comp) * n + j];
                acc.x += p.x;
                acc.y += p.y;
            }
            const double2 v = make_double2(acc.x * kInv4Pi, -acc.y * kInv4Pi);
            if (comp == 0) z[j + r * ldz] = v;
            else Z[j + (3 * r + comp - 1) * ldZ] = v;
        }
    }
}

__global__ void plane_wave_kernel(int64_t n, const double *__restrict__ px, const double *__restrict__ py,
                                  const double *__restrict__ pz, double k, double dx, double dy,
                                  double dz, double2 *__restrict__ b) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    double sn, cs;
    sincos(k * (px[i] * dx + py[i] * dy + pz[i] * dz), &sn, &cs);
    b[i] = make_double2(cs, sn);
}

// --- Krylov vector kernels (complex128, column-major) ------------------------

template <int BS>
__device__ inline double2 block_sum2(double2 v, double2 *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = BS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sh[threadIdx.x].x += sh[threadIdx.x + s].x;
            sh[threadIdx.x].y += sh[threadIdx.x + s].y;
        }
        __syncthreads();
    }
    return sh[0];
}

__global__ void zero_kernel(int64_t n, double2 *__restrict__ v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    v[i] = make_double2(0.0, 0.0);
}

// --- batched Krylov kernels ---------------------------------------------------
// The basis of right-hand side r (of R) stores vector j at V + (j R + r) n, so
// the j-th vectors of all right-hand sides form one contiguous n x R block.
// "slots" are the active right-hand sides of a launch: slot s is rhs act[s].

__global__ __launch_bounds__(kT) void bdots_kernel(int64_t n, int64_t rows_per_chunk, int k, int R,
                                                   const int32_t *__restrict__ act,
                                                   const double2 *__restrict__ V,
                                                   const double2 *__restrict__ W,
                                                   double2 *__restrict__ partial, int n_chunks) {
    __shared__ double2 sh[kT];
    const int c = blockIdx.x, j = blockIdx.y, sl = blockIdx.z;
    const int r = act[sl];
    const int64_t r0 = static_cast<int64_t>(c) * rows_per_chunk;
    const int64_t r1 = (r0 + rows_per_chunk < n) ? r0 + rows_per_chunk : n;
    const double2 *__restrict__ col = V + (static_cast<int64_t>(j) * R + r) * n;
    const double2 *__restrict__ w = W + static_cast<int64_t>(sl) * n;
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kT) {
        const double2 a = col[i], b = w[i];
        acc.x += a.x * b.x + a.y * b.y;
        acc.y += a.x * b.y - a.y * b.x;
    }
    const double2 sum = block_sum2<kT>(acc, sh);
    if (threadIdx.x == 0) partial[(static_cast<int64_t>(sl) * k + j) * n_chunks + c] = sum;
}

// h[sl * hstride + j] = sum_c partial[(sl k + j) n_chunks + c]
__global__ void bdots_final_kernel(int k, int nslots, const double2 *__restrict__ partial, int n_chunks,
                                   double2 *__restrict__ h, int hstride) {
    const int t = blockIdx.x * kT + threadIdx.x;
    if (t >= k * nslots) return;
    const int sl = t / k, j = t % k;
    double2 acc = make_double2(0.0, 0.0);
    const double2 *p = partial + (static_cast<int64_t>(sl) * k + j) * n_chunks;
    for (int c = 0; c < n_chunks; ++c) {
        acc.x += p[c].x;
        acc.y += p[c].y;
    }
    h[sl * hstride + j] = acc;
}

// W[sl] -= sum_{j<k_sl} V(j, act[sl]) h[sl * hstride + j], k_sl = min(k, kd[sl]) (kd may be null)
__global__ void bgemv_sub_kernel(int64_t n, int k, int R, const int32_t *__restrict__ act,
                                 const int32_t *__restrict__ kd, const double2 *__restrict__ V,
                                 const double2 *__restrict__ h, int hstride, double2 *__restrict__ W) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    const int sl = blockIdx.y;
    if (i >= n) return;
    const int r = act[sl];
    const int kk = kd ? (kd[sl] < k ? kd[sl] : k) : k;
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < kk; ++j) {
        const double2 a = V[(static_cast<int64_t>(j) * R + r) * n + i], b = h[sl * hstride + j];
        acc.x += a.x * b.x - a.y * b.y;
        acc.y += a.x * b.y + a.y * b.x;
    }
    double2 *w = W + static_cast<int64_t>(sl) * n;
    w[i] = make_double2(w[i].x - acc.x, w[i].y - acc.y);
}

// partial[sl * n_chunks + c] = sum over rows of chunk c of |W[sl][i]|^2
__global__ __launch_bounds__(kT) void bnorm_kernel(int64_t n, int64_t rows_per_chunk,
                                                   const double2 *__restrict__ W,
                                                   double *__restrict__ partial, int n_chunks) {
    __shared__ double2 sh[kT];
    const int c = blockIdx.x, sl = blockIdx.y;
    const int64_t r0 = static_cast<int64_t>(c) * rows_per_chunk;
    const int64_t r1 = (r0 + rows_per_chunk < n) ? r0 + rows_per_chunk : n;
    const double2 *w = W + static_cast<int64_t>(sl) * n;
    double acc = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kT) acc += w[i].x * w[i].x + w[i].y * w[i].y;
    const double2 sum = block_sum2<kT>(make_double2(acc, 0.0), sh);
    if (threadIdx.x == 0) partial[static_cast<int64_t>(sl) * n_chunks + c] = sum.x;
}

__global__ void bnorm_final_kernel(int nslots, const double *__restrict__ partial, int n_chunks,
                                   double *__restrict__ out) {
    const int sl = blockIdx.x * kT + threadIdx.x;
    if (sl >= nslots) return;
    double acc = 0.0;
    for (int c = 0; c < n_chunks; ++c) acc += partial[static_cast<int64_t>(sl) * n_chunks + c];
    out[sl] = sqrt(acc);
}

// The Gram-Schmidt update with the final sum of the projections folded in:
// every block sums the chunk partials of its slot's k coefficients (in chunk
// order, as bdots_final_kernel) into LDS, block 0 of the slot also stores them
// in h for the host, then W[sl] -= sum_j V(j, act[sl]) h_j.  k <= kFusedMaxK.
constexpr int kFusedMaxK = 1024;
// one workgroup per live right-hand side (see bblas_deflate_coef); the
// projections are staged in LDS in chunks and each thread's column loop is
// unrolled so that its loads of P and M are in flight together
__global__ __launch_bounds__(kT) void bdeflate_coef_kernel(const int32_t *__restrict__ slot,
                                                           const int32_t *__restrict__ kcount, int cs,
                                                           const double2 *__restrict__ P,
                                                           const double2 *__restrict__ M,
                                                           const double2 *__restrict__ tc, double2 *__restrict__ hc,
                                                           double2 *__restrict__ B, int col, int kb,
                                                           int64_t bstride) {
    constexpr int kChunk = 512;
    __shared__ double2 tl[kChunk];
    const int l = blockIdx.x;
    const int sl = slot[l];
    const int kc = kcount[sl];
    const double2 *t = tc + static_cast<int64_t>(l) * cs;
    const double2 *Ps = P + static_cast<int64_t>(sl) * cs * cs;
    const double2 *Ms = M + static_cast<int64_t>(sl) * cs * cs;
    // rows i = threadIdx.x + q kT, at most ceil(cs / kT) per thread
    const int rows = (cs + kT - 1) / kT;
    for (int q = 0; q < rows; ++q) {
        const int i = threadIdx.x + q * kT;
        double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
        for (int j0 = 0; j0 < kc; j0 += kChunk) {
            const int j1 = j0 + kChunk < kc ? j0 + kChunk : kc;
            __syncthreads();
            for (int j = j0 + threadIdx.x; j < j1; j += kT) tl[j - j0] = t[j];
            __syncthreads();
            if (i < cs) {
#pragma unroll 8
                for (int j = j0; j < j1; ++j) {
                    const double2 tj = tl[j - j0];
                    const double2 pv = Ps[static_cast<int64_t>(j) * cs + i];
                    const double2 mv = Ms[static_cast<int64_t>(j) * cs + i];
                    ar += pv.x * tj.x - pv.y * tj.y;
                    ai += pv.x * tj.y + pv.y * tj.x;
                    br += mv.x * tj.x - mv.y * tj.y;
                    bi += mv.x * tj.y + mv.y * tj.x;
                }
            }
        }
        if (i < cs) {
            hc[static_cast<int64_t>(l) * cs + i] = i < kc ? make_double2(ar, ai) : make_double2(0.0, 0.0);
            if (i + 1 < kc) {
                double2 *b = B + static_cast<int64_t>(sl) * bstride + static_cast<int64_t>(col) * kb + i;
                *b = make_double2(b->x + br, b->y + bi);
            }
        }
    }
}

__global__ __launch_bounds__(kT) void bgemv_sub_partial_kernel(int64_t n, int k, int R, const int32_t *__restrict__ act,
                                                               const double2 *__restrict__ V,
                                                               const double2 *__restrict__ partial, int n_chunks,
                                                               double2 *__restrict__ h, int hstride,
                                                               double2 *__restrict__ W) {
    __shared__ double2 hc[kFusedMaxK];
    const int sl = blockIdx.y;
    for (int j = threadIdx.x; j < k; j += kT) {
        double2 acc = make_double2(0.0, 0.0);
        const double2 *p = partial + (static_cast<int64_t>(sl) * k + j) * n_chunks;
        for (int c = 0; c < n_chunks; ++c) {
            acc.x += p[c].x;
            acc.y += p[c].y;
        }
        hc[j] = acc;
        if (blockIdx.x == 0) h[sl * hstride + j] = acc;
    }
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    const int r = act[sl];
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < k; ++j) {
        const double2 a = V[(static_cast<int64_t>(j) * R + r) * n + i], b = hc[j];
        acc.x += a.x * b.x - a.y * b.y;
        acc.y += a.x * b.y + a.y * b.x;
    }
    double2 *w = W + static_cast<int64_t>(sl) * n;
    w[i] = make_double2(w[i].x - acc.x, w[i].y - acc.y);
}

// The new basis vector with the final sum of the norm folded in: every block
// sums its slot's chunk partials (in chunk order, as bnorm_final_kernel),
// block 0 of the slot stores the norm for the host, then
// V(kcol, act[sl]) = W[sl] / nrm (zero when nrm == 0).
__global__ __launch_bounds__(kT) void bnorm_scale_kernel(int64_t n, int kcol, int R, const int32_t *__restrict__ act,
                                                         const double2 *__restrict__ W,
                                                         const double *__restrict__ partial, int n_chunks,
                                                         double *__restrict__ nrm, double2 *__restrict__ V) {
    __shared__ double snrm;
    const int sl = blockIdx.y;
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int c = 0; c < n_chunks; ++c) acc += partial[static_cast<int64_t>(sl) * n_chunks + c];
        snrm = sqrt(acc);
        if (blockIdx.x == 0) nrm[sl] = snrm;
    }
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    const double sc = snrm;
    const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
    const double2 w = W[static_cast<int64_t>(sl) * n + i];
    V[(static_cast<int64_t>(kcol) * R + act[sl]) * n + i] = make_double2(w.x * inv, w.y * inv);
}

// V(kcol, act[sl]) = W[sl] / nrm[sl]   (zero when nrm[sl] == 0)
__global__ void bscale_into_basis_kernel(int64_t n, int kcol, int R, const int32_t *__restrict__ act,
                                         const double2 *__restrict__ W, const double *__restrict__ nrm,
                                         double2 *__restrict__ V) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    const int sl = blockIdx.y;
    if (i >= n) return;
    const double s = nrm[sl];
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    const double2 w = W[static_cast<int64_t>(sl) * n + i];
    V[(static_cast<int64_t>(kcol) * R + act[sl]) * n + i] = make_double2(w.x * inv, w.y * inv);
}

// X[sl] = src[act[sl] * ld + i]  (gather columns of a column-major block)
__global__ void bgather_kernel(int64_t n, const int32_t *__restrict__ act,
                               const double2 *__restrict__ src, int64_t ld, double2 *__restrict__ X) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    const int sl = blockIdx.y;
    if (i >= n) return;
    X[static_cast<int64_t>(sl) * n + i] = src[static_cast<int64_t>(act[sl]) * ld + i];
}

// x[act[sl] * ldx + i] += sum_{j < kd[sl]} V(j, act[sl]) y[sl * ystride + j]
__global__ void bupdate_kernel(int64_t n, int R, const int32_t *__restrict__ act,
                               const int32_t *__restrict__ kd, const double2 *__restrict__ V,
                               const double2 *__restrict__ y, int ystride, double2 *__restrict__ x,
                               int64_t ldx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    const int sl = blockIdx.y;
    if (i >= n) return;
    const int r = act[sl];
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < kd[sl]; ++j) {
        const double2 a = V[(static_cast<int64_t>(j) * R + r) * n + i], b = y[sl * ystride + j];
        acc.x += a.x * b.x - a.y * b.y;
        acc.y += a.x * b.y + a.y * b.x;
    }
    double2 *xc = x + static_cast<int64_t>(r) * ldx;
    xc[i] = make_double2(xc[i].x + acc.x, xc[i].y + acc.y);
}

// out[sl] = b[act[sl]] - ax[sl]   (ax and out hold slots contiguously)
__global__ void bsub_kernel(int64_t n, const int32_t *__restrict__ act, const double2 *__restrict__ b,
                            int64_t ldb, const double2 *__restrict__ ax, double2 *__restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    const int sl = blockIdx.y;
    if (i >= n) return;
    const double2 bv = b[static_cast<int64_t>(act[sl]) * ldb + i];
    const double2 av = ax[static_cast<int64_t>(sl) * n + i];
    out[static_cast<int64_t>(sl) * n + i] = make_double2(bv.x - av.x, bv.y - av.y);
}

// x[act[sl] * ldx + i] += W[sl * n + i]
__global__ void scatter_add_kernel(int64_t n, const int32_t *__restrict__ act, const double2 *__restrict__ W,
                                   double2 *__restrict__ x, int64_t ldx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    const int sl = blockIdx.y;
    if (i >= n) return;
    const double2 w = W[static_cast<int64_t>(sl) * n + i];
    double2 *xc = x + static_cast<int64_t>(act[sl]) * ldx;
    xc[i] = make_double2(xc[i].x + w.x, xc[i].y + w.y);
}

// C[j * ldc + i] = sum over slabs t (in order) of P[t * cnt + j * m + i], cnt = m * nn
__global__ void sum_slabs_kernel(int64_t m, int64_t cnt, int parts, const double2 *__restrict__ P,
                                 double2 *__restrict__ C, int64_t ldc) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (e >= cnt) return;
    double sx = 0.0, sy = 0.0;
    for (int t = 0; t < parts; ++t) {
        const double2 v = P[static_cast<int64_t>(t) * cnt + e];
        sx += v.x;
        sy += v.y;
    }
    const int64_t j = e / m, i = e - j * m;
    C[j * ldc + i] = make_double2(sx, sy);
}

// Tall-skinny block products of block GMRES for blocks of at most
// kTsMaxCols columns (the Gram-Schmidt projections V^H W and updates
// W -= V H, CholeskyQR's Gram matrices and W T^{-1}, the deflation).  n is
// long (the unknowns), the other two sizes are small, and the operands are
// column-major.  Both products are bound by reading the tall operand once.
//
// ts_cn_kernel: slab partials of C = A^H B, A rows x m, B rows x nn
// (nn <= 8 NQ).  Workgroup (slab, tile) takes 32 columns of A and every
// column of B over the rows of its slab, 32 rows at a time staged in LDS
// (each column's 32 rows are one 512-byte read); thread t owns A column
// t % 32 of the tile and B columns t / 32 + 8 u.  The partials go to
// P[slab][r][j] (an m x nn column-major block per slab) and are added in slab
// order by sum_slabs_kernel.
constexpr int kTsTile = 32;

template <int NQ>
__global__ __launch_bounds__(kT) void ts_cn_kernel(int64_t rows, int m, int nn, const double2 *__restrict__ A,
                                                   int64_t lda, const double2 *__restrict__ B, int64_t ldb,
                                                   int64_t slab_rows, double2 *__restrict__ P) {
    __shared__ double2 sa[kTsTile][kTsTile + 1];
    __shared__ double2 sb[kTsTile][8 * NQ + 1];
    const int t = threadIdx.x, j = t & 31, q = t >> 5, i = t & 31;
    const int j0 = blockIdx.y * kTsTile;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * slab_rows;
    const int64_t r1 = r0 + slab_rows < rows ? r0 + slab_rows : rows;
    double ar[NQ], ai[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) ar[u] = ai[u] = 0.0;
    for (int64_t base = r0; base < r1; base += kTsTile) {
        const int len = static_cast<int>(r1 - base < kTsTile ? r1 - base : kTsTile);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = q + 8 * u;
            double2 v = make_double2(0.0, 0.0);
            if (i < len && j0 + c < m) v = A[static_cast<int64_t>(j0 + c) * lda + base + i];
            sa[i][c] = v;
        }
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int c = q + 8 * u;
            double2 v = make_double2(0.0, 0.0);
            if (i < len && c < nn) v = B[static_cast<int64_t>(c) * ldb + base + i];
            sb[i][c] = v;
        }
        __syncthreads();
        // rows past the slab's end were staged as zeros
#pragma unroll 8
        for (int ii = 0; ii < kTsTile; ++ii) {
            const double2 a = sa[ii][j];
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const double2 b = sb[ii][q + 8 * u];
                // conj(a) b
                ar[u] = fma(a.x, b.x, fma(a.y, b.y, ar[u]));
                ai[u] = fma(a.x, b.y, fma(-a.y, b.x, ai[u]));
            }
        }
        __syncthreads();
    }
    double2 *Ps = P + static_cast<int64_t>(blockIdx.x) * m * nn;
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int r = q + 8 * u;
        if (j0 + j < m && r < nn) Ps[static_cast<int64_t>(r) * m + j0 + j] = make_double2(ar[u], ai[u]);
    }
}

// ts_nn_kernel: C = alpha A B (+ C when accumulate), A rows x k, B k x nn
// (nn <= 8 NQ, on the device), C rows x nn.  One thread per row keeps the
// row's nn sums; B is staged 64 rows at a time in LDS and read as broadcasts.
template <int NQ>
__global__ __launch_bounds__(kT) void ts_nn_kernel(int64_t rows, int k, int nn, double alpha, int accumulate,
                                                   const double2 *__restrict__ A, int64_t lda,
                                                   const double2 *__restrict__ B, int64_t ldb,
                                                   double2 *__restrict__ C, int64_t ldc) {
    constexpr int NC = 8 * NQ;
    __shared__ double2 sb[64][NC];
    const int t = threadIdx.x;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + t;
    double cr[NC], ci[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) cr[r] = ci[r] = 0.0;
    for (int j0 = 0; j0 < k; j0 += 64) {
        const int len = k - j0 < 64 ? k - j0 : 64;
        __syncthreads();
        for (int e = t; e < 64 * NC; e += kT) {
            const int jj = e & 63, r = e >> 6;
            sb[jj][r] = (jj < len && r < nn) ? B[static_cast<int64_t>(r) * ldb + j0 + jj] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (i < rows) {
            const double2 *Ac = A + static_cast<int64_t>(j0) * lda + i;
#pragma unroll 4
            for (int jj = 0; jj < len; ++jj) {
                const double2 a = Ac[static_cast<int64_t>(jj) * lda];
#pragma unroll
                for (int r = 0; r < NC; ++r) {
                    const double2 b = sb[jj][r];
                    cr[r] = fma(a.x, b.x, fma(-a.y, b.y, cr[r]));
                    ci[r] = fma(a.x, b.y, fma(a.y, b.x, ci[r]));
                }
            }
        }
    }
    if (i >= rows) return;
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        if (r < nn) {
            double2 *c = C + static_cast<int64_t>(r) * ldc + i;
            double2 v = make_double2(alpha * cr[r], alpha * ci[r]);
            if (accumulate) {
                const double2 o = *c;
                v.x += o.x;
                v.y += o.y;
            }
            *c = v;
        }
    }
}

// The same sum for many slabs (the tall-skinny products' partials: a few
// hundred slabs of a small block): a workgroup takes 16 outputs, its 16 groups
// of 16 threads add every 16th slab (consecutive outputs, so each load is one
// 256-byte run), and the group sums are added in group order in LDS.
__global__ __launch_bounds__(kT) void sum_slabs_grouped_kernel(int64_t m, int64_t cnt, int parts,
                                                               const double2 *__restrict__ P,
                                                               double2 *__restrict__ C, int64_t ldc) {
    __shared__ double2 part[16][17];
    const int t = threadIdx.x, o = t & 15, g = t >> 4;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 16 + o;
    double sx = 0.0, sy = 0.0;
    if (e < cnt) {
#pragma unroll 4
        for (int q = g; q < parts; q += 16) {
            const double2 v = P[static_cast<int64_t>(q) * cnt + e];
            sx += v.x;
            sy += v.y;
        }
    }
    part[g][o] = make_double2(sx, sy);
    __syncthreads();
    if (g == 0 && e < cnt) {
        for (int q = 1; q < 16; ++q) {
            sx += part[q][o].x;
            sy += part[q][o].y;
        }
        const int64_t j = e / m, i = e - j * m;
        C[j * ldc + i] = make_double2(sx, sy);
    }
}

// Cholesky factor of a small Hermitian Gram matrix G = T^H T (r x r,
// column-major, r <= kSmallChol), T upper triangular, in one workgroup: the
// right-looking (outer-product) form, one pivot per step.  As the host
// factorisation of block GMRES: a diagonal shift (0, then 1e-14 dmax, times
// 100 up to 1e-4 dmax, dmax the largest diagonal entry) is added only when a
// pivot is not safely positive.  Writes T, Ti = T^{-1} and, when Tprev is
// given, Tout = T Tprev (all r x r column-major); status 0 on success, 1 for
// a zero or non-finite block, 2 when no shift gives a positive factor (then
// nothing else is written).
__global__ __launch_bounds__(256) void small_chol_kernel(const double2 *__restrict__ G, int r,
                                                         double2 *__restrict__ T, double2 *__restrict__ Ti,
                                                         const double2 *__restrict__ Tprev,
                                                         double2 *__restrict__ Tout, int *__restrict__ status) {
    __shared__ double2 A[kSmallChol * kSmallChol];
    __shared__ double2 U[kSmallChol * kSmallChol];
    __shared__ int ok;
    __shared__ double dmax_s;
    const int tid = threadIdx.x, nt = blockDim.x, rr = r * r;
    if (tid == 0) {
        double d = 0.0;
        for (int i = 0; i < r; ++i) d = fmax(d, G[i * r + i].x);
        dmax_s = d;
    }
    __syncthreads();
    const double dmax = dmax_s;
    if (!(dmax > 0.0) || !isfinite(dmax)) {
        if (tid == 0) *status = 1;
        return;
    }
    for (double shift = 0.0;; shift = shift == 0.0 ? 1e-14 * dmax : shift * 100.0) {
        if (shift > 1e-4 * dmax) {
            if (tid == 0) *status = 2;
            return;
        }
        for (int e = tid; e < rr; e += nt) {
            A[e] = G[e];
            U[e] = make_double2(0.0, 0.0);
        }
        if (tid == 0) ok = 1;
        __syncthreads();
        for (int k = 0; k < r; ++k) {
            if (tid == 0) {
                const double akk = A[k * r + k].x + shift;
                if (akk > 1e-15 * dmax) U[k * r + k] = make_double2(sqrt(akk), 0.0);
                else ok = 0;
            }
            __syncthreads();
            if (!ok) break;
            const double ukk = U[k * r + k].x;
            for (int j = k + 1 + tid; j < r; j += nt) {  // row k: U(k, j) = A(k, j) / U(k, k)
                const double2 a = A[j * r + k];
                U[j * r + k] = make_double2(a.x / ukk, a.y / ukk);
            }
            __syncthreads();
            for (int e = tid; e < rr; e += nt) {  // A(i, j) -= conj(U(k, i)) U(k, j), k < i <= j
                const int j = e / r, i = e - j * r;
                if (i > k && i <= j) {
                    const double2 ui = U[i * r + k], uj = U[j * r + k];
                    A[e].x -= ui.x * uj.x + ui.y * uj.y;
                    A[e].y -= ui.x * uj.y - ui.y * uj.x;
                }
            }
            __syncthreads();
        }
        if (ok) break;
        __syncthreads();
    }
    for (int e = tid; e < rr; e += nt) T[e] = U[e];
    if (tid < r) {  // column j of T^{-1} by back substitution (into A, no longer needed)
        const int j = tid;
        double2 *x = A + j * r;
        for (int i = j; i >= 0; --i) {
            double sx = i == j ? 1.0 : 0.0, sy = 0.0;
            for (int m = i + 1; m <= j; ++m) {
                const double2 u = U[m * r + i];
                sx -= u.x * x[m].x - u.y * x[m].y;
                sy -= u.x * x[m].y + u.y * x[m].x;
            }
            const double d = U[i * r + i].x;
            x[i] = make_double2(sx / d, sy / d);
        }
        for (int i = 0; i < r; ++i) Ti[j * r + i] = i <= j ? x[i] : make_double2(0.0, 0.0);
    }
    if (Tprev) {
        for (int e = tid; e < rr; e += nt) {  // Tout(i, j) = sum_{i <= m <= j} U(i, m) Tprev(m, j)
            const int j = e / r, i = e - j * r;
            double sx = 0.0, sy = 0.0;
            for (int m = i; m <= j; ++m) {
                const double2 u = U[m * r + i], t = Tprev[j * r + m];
                sx += u.x * t.x - u.y * t.y;
                sy += u.x * t.y + u.y * t.x;
            }
            Tout[e] = make_double2(sx, sy);
        }
    }
    if (tid == 0) *status = 0;
}

}  // namespace

#define LAUNCH_CHECK() VSIE_HIP(hipGetLastError())

void launch_weights(const DeviceMesh &m, const double *k0, int n_freq, hipStream_t s) {
    if (m.n == 0) return;
    hipLaunchKernelGGL(weights_kernel, dim3(blocks_for(m.n)), dim3(kT), 0, s, m, k0, n_freq);
    LAUNCH_CHECK();
}

void launch_pack_charges(SrcClass cls, vsie_precision prec, const SourceSet &src,
                         const double *sp_f, int nrhs, const double2 *x, int64_t ldx,
                         bool conj_in, void *charge, hipStream_t s) {
    if (src.count == 0) return;
    const double *sc = (cls == kClassG) ? sp_f : nullptr;
    if (prec == VSIE_FP64)
        hipLaunchKernelGGL(pack_kernel<double2>, dim3(blocks_for(src.count)), dim3(kT), 0, s,
                           src.count, src.idx, sc, nrhs, x, ldx, conj_in,
                           static_cast<double2 *>(charge));
    else
        hipLaunchKernelGGL(pack_kernel<float2>, dim3(blocks_for(src.count)), dim3(kT), 0, s,
                           src.count, src.idx, sc, nrhs, x, ldx, conj_in,
                           static_cast<float2 *>(charge));
    LAUNCH_CHECK();
}

void launch_pack_both(vsie_precision prec, const SourceSet &G, const SourceSet &F, const double *sp_f, int nrhs,
                      const double2 *x, int64_t ldx, bool conj_in, void *chargeG, void *chargeF, hipStream_t s) {
    const int64_t total = G.count + F.count;
    if (total == 0) return;
    if (prec == VSIE_FP64)
        hipLaunchKernelGGL(pack2_kernel<double2>, dim3(blocks_for(total)), dim3(kT), 0, s, G.count, G.idx, sp_f,
                           F.count, F.idx, nrhs, x, ldx, conj_in, static_cast<double2 *>(chargeG),
                           static_cast<double2 *>(chargeF));
    else
        hipLaunchKernelGGL(pack2_kernel<float2>, dim3(blocks_for(total)), dim3(kT), 0, s, G.count, G.idx, sp_f,
                           F.count, F.idx, nrhs, x, ldx, conj_in, static_cast<float2 *>(chargeG),
                           static_cast<float2 *>(chargeF));
    LAUNCH_CHECK();
}

void launch_pack_plain(vsie_precision prec, int64_t n, int nrhs, const double2 *x, int64_t ldx,
                       bool conj_in, void *charge, hipStream_t s) {
    if (n == 0) return;
    if (prec == VSIE_FP64)
        hipLaunchKernelGGL(pack_kernel<double2>, dim3(blocks_for(n)), dim3(kT), 0, s, n,
                           static_cast<const int32_t *>(nullptr), static_cast<const double *>(nullptr),
                           nrhs, x, ldx, conj_in, static_cast<double2 *>(charge));
    else
        hipLaunchKernelGGL(pack_kernel<float2>, dim3(blocks_for(n)), dim3(kT), 0, s, n,
                           static_cast<const int32_t *>(nullptr), static_cast<const double *>(nullptr),
                           nrhs, x, ldx, conj_in, static_cast<float2 *>(charge));
    LAUNCH_CHECK();
}

void launch_reduce_partials(int64_t n_t, int nrhs, int n_parts, const double2 *partial,
                            const double2 *diag, bool conj_diag, const double2 *x, int64_t ldx,
                            double2 *y, int64_t ldy, double2 *, hipStream_t s) {
    if (n_t == 0) return;
    hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(n_t)), dim3(kT), 0, s, n_t, nrhs, n_parts,
                       partial, diag, conj_diag, x, ldx, y, ldy);
    LAUNCH_CHECK();
}

void launch_pack_planar(int64_t n, int nrhs, const double2 *x, int64_t ldx, float *X2, hipStream_t s) {
    if (n == 0 || nrhs == 0) return;
    hipLaunchKernelGGL(pack_planar_kernel, dim3(blocks_for(n), nrhs), dim3(kT), 0, s, n, nrhs, x, ldx, X2);
    LAUNCH_CHECK();
}

void launch_reduce_planar(int64_t n, int nrhs, int n_parts, const float *partial, const double2 *diag,
                          bool adjoint, const double2 *x, int64_t ldx, double2 *y, int64_t ldy, hipStream_t s) {
    if (n == 0 || nrhs == 0) return;
    hipLaunchKernelGGL(reduce_planar_kernel, dim3(blocks_for(n), nrhs), dim3(kT), 0, s, n, nrhs, n_parts,
                       partial, diag, adjoint, x, ldx, y, ldy);
    LAUNCH_CHECK();
}

void launch_scatter_conj(int64_t count, const int32_t *idx, const double *sp, int nrhs,
                         int n_parts, const double2 *partial, double2 *y, int64_t ldy,
                         hipStream_t s) {
    if (count == 0) return;
    hipLaunchKernelGGL(scatter_conj_kernel, dim3(blocks_for(count)), dim3(kT), 0, s, count, idx, sp,
                       nrhs, n_parts, partial, y, ldy);
    LAUNCH_CHECK();
}

void launch_sums_reduce(int64_t n, int nrhs, int n_parts, const double2 *partial, double2 *z,
                        int64_t ldz, double2 *Z, int64_t ldZ, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(sums_reduce_kernel, dim3(blocks_for(n)), dim3(kT), 0, s, n, nrhs, n_parts,
                       partial, z, ldz, Z, ldZ);
    LAUNCH_CHECK();
}

void launch_plane_wave(int64_t n, const double *px, const double *py, const double *pz, double k,
                       double dx, double dy, double dz, double2 *b, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(plane_wave_kernel, dim3(blocks_for(n)), dim3(kT), 0, s, n, px, py, pz, k,
                       dx, dy, dz, b);
    LAUNCH_CHECK();
}

void blas_zero(int64_t n, double2 *v, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(n)), dim3(kT), 0, s, n, v);
    LAUNCH_CHECK();
}

}  // namespace vsie

namespace vsie {

static int64_t rpc(int64_t n, int n_chunks) { return (n + n_chunks - 1) / n_chunks; }

void bblas_dots(int64_t n, int k, int R, int nslots, const int32_t *act, const double2 *V,
                const double2 *W, double2 *partial, int n_chunks, double2 *h, int hstride,
                hipStream_t s) {
    if (k == 0 || nslots == 0) return;
    hipLaunchKernelGGL(bdots_kernel, dim3(n_chunks, k, nslots), dim3(kT), 0, s, n, rpc(n, n_chunks), k,
                       R, act, V, W, partial, n_chunks);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(bdots_final_kernel, dim3(blocks_for(static_cast<int64_t>(k) * nslots)), dim3(kT),
                       0, s, k, nslots, partial, n_chunks, h, hstride);
    LAUNCH_CHECK();
}

void bblas_gemv_sub(int64_t n, int k, int R, int nslots, const int32_t *act, const double2 *V,
                    const double2 *h, int hstride, double2 *W, hipStream_t s, const int32_t *kd) {
    if (k == 0 || nslots == 0) return;
    hipLaunchKernelGGL(bgemv_sub_kernel, dim3(blocks_for(n), nslots), dim3(kT), 0, s, n, k, R, act, kd,
                       V, h, hstride, W);
    LAUNCH_CHECK();
}

void bblas_norm(int64_t n, int nslots, const double2 *W, double *partial, int n_chunks, double *out,
                hipStream_t s) {
    if (nslots == 0) return;
    hipLaunchKernelGGL(bnorm_kernel, dim3(n_chunks, nslots), dim3(kT), 0, s, n, rpc(n, n_chunks), W,
                       partial, n_chunks);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(bnorm_final_kernel, dim3(blocks_for(nslots)), dim3(kT), 0, s, nslots, partial,
                       n_chunks, out);
    LAUNCH_CHECK();
}

bool bblas_fused_ok(int k) { return k <= kFusedMaxK; }

void bblas_dots_partial(int64_t n, int k, int R, int nslots, const int32_t *act, const double2 *V,
                        const double2 *W, double2 *partial, int n_chunks, hipStream_t s) {
    if (k == 0 || nslots == 0) return;
    hipLaunchKernelGGL(bdots_kernel, dim3(n_chunks, k, nslots), dim3(kT), 0, s, n, rpc(n, n_chunks), k,
                       R, act, V, W, partial, n_chunks);
    LAUNCH_CHECK();
}

void bblas_deflate_coef(int nl, const int32_t *slot, const int32_t *kcount, int cs, const double2 *P,
                        const double2 *M, const double2 *tc, double2 *hc, double2 *B, int col, int kb,
                        int64_t bstride, hipStream_t s) {
    if (nl == 0) return;
    hipLaunchKernelGGL(bdeflate_coef_kernel, dim3(nl), dim3(kT), 0, s, slot, kcount, cs, P, M, tc, hc, B, col, kb,
                       bstride);
    LAUNCH_CHECK();
}

void bblas_gemv_sub_partial(int64_t n, int k, int R, int nslots, const int32_t *act, const double2 *V,
                            const double2 *partial, int n_chunks, double2 *h, int hstride, double2 *W,
                            hipStream_t s) {
    if (k == 0 || nslots == 0) return;
    if (k > kFusedMaxK) fail(VSIE_E_INVALID, "fused Gram-Schmidt update: too many basis vectors");
    hipLaunchKernelGGL(bgemv_sub_partial_kernel, dim3(blocks_for(n), nslots), dim3(kT), 0, s, n, k, R, act, V,
                       partial, n_chunks, h, hstride, W);
    LAUNCH_CHECK();
}

void bblas_norm_partial(int64_t n, int nslots, const double2 *W, double *partial, int n_chunks, hipStream_t s) {
    if (nslots == 0) return;
    hipLaunchKernelGGL(bnorm_kernel, dim3(n_chunks, nslots), dim3(kT), 0, s, n, rpc(n, n_chunks), W,
                       partial, n_chunks);
    LAUNCH_CHECK();
}

void bblas_norm_scale(int64_t n, int kcol, int R, int nslots, const int32_t *act, const double2 *W,
                      const double *partial, int n_chunks, double *nrm, double2 *V, hipStream_t s) {
    if (nslots == 0) return;
    hipLaunchKernelGGL(bnorm_scale_kernel, dim3(blocks_for(n), nslots), dim3(kT), 0, s, n, kcol, R, act, W,
                       partial, n_chunks, nrm, V);
    LAUNCH_CHECK();
}

void bblas_scale_into_basis(int64_t n, int kcol, int R, int nslots, const int32_t *act,
                            const double2 *W, const double *nrm, double2 *V, hipStream_t s) {
    if (nslots == 0) return;
    hipLaunchKernelGGL(bscale_into_basis_kernel, dim3(blocks_for(n), nslots), dim3(kT), 0, s, n, kcol, R,
                       act, W, nrm, V);
    LAUNCH_CHECK();
}

void bblas_gather(int64_t n, int nslots, const int32_t *act, const double2 *src, int64_t ld,
                  double2 *X, hipStream_t s) {
    if (nslots == 0) return;
    hipLaunchKernelGGL(bgather_kernel, dim3(blocks_for(n), nslots), dim3(kT), 0, s, n, act, src, ld, X);
    LAUNCH_CHECK();
}

void bblas_update(int64_t n, int R, int nslots, const int32_t *act, const int32_t *kd, const double2 *V,
                  const double2 *y, int ystride, double2 *x, int64_t ldx, hipStream_t s) {
    if (nslots == 0) return;
    hipLaunchKernelGGL(bupdate_kernel, dim3(blocks_for(n), nslots), dim3(kT), 0, s, n, R, act, kd, V, y,
                       ystride, x, ldx);
    LAUNCH_CHECK();
}

void bblas_sub(int64_t n, int nslots, const int32_t *act, const double2 *b, int64_t ldb,
               const double2 *ax, double2 *out, hipStream_t s) {
    if (nslots == 0) return;
    hipLaunchKernelGGL(bsub_kernel, dim3(blocks_for(n), nslots), dim3(kT), 0, s, n, act, b, ldb, ax, out);
    LAUNCH_CHECK();
}

}  // namespace vsie

namespace vsie {
void blas_scatter_add(int64_t n, int nslots, const int32_t *act, const double2 *W, double2 *x, int64_t ldx,
                      hipStream_t s) {
    if (nslots == 0 || n == 0) return;
    hipLaunchKernelGGL(scatter_add_kernel, dim3(blocks_for(n), nslots), dim3(kT), 0, s, n, act, W, x, ldx);
    LAUNCH_CHECK();
}

void launch_small_chol(const double2 *G, int r, double2 *T, double2 *Ti, const double2 *Tprev, double2 *Tout,
                       int *status, hipStream_t s) {
    if (r < 1 || r > kSmallChol) fail(VSIE_E_INVALID, "small Cholesky: block width out of range");
    hipLaunchKernelGGL(small_chol_kernel, dim3(1), dim3(256), 0, s, G, r, T, Ti, Tprev, Tout, status);
    LAUNCH_CHECK();
}

// Rows per slab of ts_cn: about 2048 workgroups over the slabs and 32-column
// tiles, at least 256 rows (8 staged tiles) per slab, a multiple of 32.
int64_t ts_cn_slab_rows(int64_t m, int64_t rows) {
    const int64_t tiles = (m + kTsTile - 1) / kTsTile;
    int64_t slabs = (2048 + tiles - 1) / tiles;
    slabs = std::max<int64_t>(1, std::min(slabs, rows / 256));
    const int64_t sr = (rows + slabs - 1) / slabs;
    return std::max<int64_t>(kTsTile, (sr + kTsTile - 1) / kTsTile * kTsTile);
}

size_t ts_cn_bytes(int64_t m, int64_t nn, int64_t rows) {
    if (rows <= 0) return 0;
    const int64_t sr = ts_cn_slab_rows(m, rows);
    return sizeof(double2) * static_cast<size_t>(m * nn * ((rows + sr - 1) / sr));
}

void ts_cn(int64_t rows, int64_t m, int64_t nn, const double2 *A, int64_t lda, const double2 *B, int64_t ldb,
           double2 *P, double2 *C, int64_t ldc, hipStream_t s) {
    if (m <= 0 || nn <= 0) return;
    if (rows < 1 || nn > kTsMaxCols || m > INT32_MAX || lda < rows || ldb < rows || ldc < m)
        fail(VSIE_E_INVALID, "tall-skinny product: operand shapes out of range");
    const int64_t sr = ts_cn_slab_rows(m, rows);
    const int64_t slabs = (rows + sr - 1) / sr;
    const int64_t tiles = (m + kTsTile - 1) / kTsTile;
    if (slabs > 0x7fffffff || tiles > 65535) fail(VSIE_E_INVALID, "tall-skinny product: grid too large");
    const dim3 grid(static_cast<unsigned>(slabs), static_cast<unsigned>(tiles));
    const int mi = static_cast<int>(m), ni = static_cast<int>(nn);
    if (nn <= 8) hipLaunchKernelGGL(ts_cn_kernel<1>, grid, dim3(kT), 0, s, rows, mi, ni, A, lda, B, ldb, sr, P);
    else if (nn <= 16) hipLaunchKernelGGL(ts_cn_kernel<2>, grid, dim3(kT), 0, s, rows, mi, ni, A, lda, B, ldb, sr, P);
    else hipLaunchKernelGGL(ts_cn_kernel<4>, grid, dim3(kT), 0, s, rows, mi, ni, A, lda, B, ldb, sr, P);
    LAUNCH_CHECK();
    blas_sum_slabs(m, nn, static_cast<int>(slabs), P, C, ldc, s);
}

void ts_nn(int64_t rows, int64_t k, int64_t nn, double alpha, bool accumulate, const double2 *A, int64_t lda,
           const double2 *B, int64_t ldb, double2 *C, int64_t ldc, hipStream_t s) {
    if (rows <= 0 || nn <= 0) return;
    if (nn > kTsMaxCols || k > INT32_MAX || (k > 0 && (lda < rows || ldb < k)) || ldc < rows)
        fail(VSIE_E_INVALID, "tall-skinny product: operand shapes out of range");
    const unsigned blocks = blocks_for(rows);
    const int ki = static_cast<int>(k), ni = static_cast<int>(nn), acc = accumulate ? 1 : 0;
    if (nn <= 8) hipLaunchKernelGGL(ts_nn_kernel<1>, dim3(blocks), dim3(kT), 0, s, rows, ki, ni, alpha, acc, A, lda, B, ldb, C, ldc);
    else if (nn <= 16) hipLaunchKernelGGL(ts_nn_kernel<2>, dim3(blocks), dim3(kT), 0, s, rows, ki, ni, alpha, acc, A, lda, B, ldb, C, ldc);
    else hipLaunchKernelGGL(ts_nn_kernel<4>, dim3(blocks), dim3(kT), 0, s, rows, ki, ni, alpha, acc, A, lda, B, ldb, C, ldc);
    LAUNCH_CHECK();
}

void blas_sum_slabs(int64_t m, int64_t nn, int parts, const double2 *P, double2 *C, int64_t ldc, hipStream_t s) {
    const int64_t cnt = m * nn;
    if (cnt == 0) return;
    if (parts > 16)
        hipLaunchKernelGGL(sum_slabs_grouped_kernel, dim3(blocks_for(cnt, 16)), dim3(kT), 0, s, m, cnt, parts, P, C,
                           ldc);
    else
        hipLaunchKernelGGL(sum_slabs_kernel, dim3(blocks_for(cnt)), dim3(kT), 0, s, m, cnt, parts, P, C, ldc);
    LAUNCH_CHECK();
}
}  // namespace vsie
