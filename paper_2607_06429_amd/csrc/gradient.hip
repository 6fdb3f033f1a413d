// Adjoint-state gradient of a receiver misfit with respect to per-cell sound
// speed and density.
//
// With A p = b (the collocation system of the final VSIE, Theorem 3), receiver
// pressures p_rec = p_inc - E p where E_rj = -A(x_r, j) is the off-diagonal
// kernel at receiver points (the representation formula of section 2.3.1),
// and a real misfit J(p_rec) whose conjugate-Wirtinger gradient is rho_r:
//
//   adjoint system   A^H lam = E^H rho,   (E^H rho)_j = s_j zR_j - v_j . ZR_j
//   dJ = Re sum_q [ rho^H dE p - lam^H dA p ]
//
// which, per element j and right-hand side q, gives (z, Z from the adjoint
// solution lam over collocation targets, zR, ZR from rho over receivers)
//   dJ/ds_j = Re p_j ( conj zR_j + conj z_j + conj lam_j S_j / |cell_j| )
//   dJ/dv_j = -Re p_j ( conj ZR_j + conj Z_j )
//   dJ/dm_j = -Re conj(lam_j) p_j
// and the chain rule to (c_k, rho_k) through
//   s_k = |cell| (rho0/rho_k) k0^2 ((c0/c_k)^2 - 1),  m_k = rho0/rho_k,
//   faces: m_f = (rho0/rho_in + rho0/rho_out)/2,  v_f = -|face| (alpha_in - alpha_out) n_f,
//   cells: v_j = |cell| grad alpha_j from the same-subdomain neighbour stencil,
//   alpha = rho0/rho - 1.
#include "vsie_internal.h"

namespace vsie {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr int kT = 256;

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kT - 1) / kT); }

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Same integral as the weights use (duplicated here to keep the translation
// units independent): integral of G over the ball of radius a centred at 0.
__device__ double2 ball_integral(double a, double k) {
    const double ka = k * a;
    if (ka < 0.5) {
        double2 t = make_double2(-0.5 * ka * ka, 0.0);
        double2 acc = make_double2(-t.x, -t.y);
        for (int n = 3; n < 30; ++n) {
            t = cmul(t, make_double2(0.0, ka / n));
            acc.x += (1 - n) * t.x;
            acc.y += (1 - n) * t.y;
        }
        return make_double2(acc.x / (k * k), acc.y / (k * k));
    }
    double sn, cs;
    sincos(ka, &sn, &cs);
    return make_double2((cs + ka * sn - 1.0) / (k * k), (sn - ka * cs) / (k * k));
}

// out_j = s_j zR_j - v_j . ZR_j  (s = 4 pi s', v = 4 pi v')
__global__ void adjoint_rhs_kernel(int64_t n, int nrhs, const double *__restrict__ sp,
                                   const double *__restrict__ vpx, const double *__restrict__ vpy,
                                   const double *__restrict__ vpz, const double2 *__restrict__ zR,
                                   int64_t ldz, const double2 *__restrict__ ZR, int64_t ldZ,
                                   double2 *__restrict__ out, int64_t ldo) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (j >= n) return;
    const double s = 4.0 * kPi * sp[j];
    const double v[3] = {4.0 * kPi * vpx[j], 4.0 * kPi * vpy[j], 4.0 * kPi * vpz[j]};
    for (int q = 0; q < nrhs; ++q) {
        const double2 a = zR[j + q * ldz];
        double2 acc = make_double2(s * a.x, s * a.y);
        for (int ax = 0; ax < 3; ++ax) {
            const double2 b = ZR[j + (3 * q + ax) * ldZ];
            acc.x -= v[ax] * b.x;
            acc.y -= v[ax] * b.y;
        }
        out[j + q * ldo] = acc;
    }
}

struct SensArgs {
    int64_t n, n_vol;
    int nrhs;
    double k;
    const double *vw;
    const double2 *P;
    int64_t ldp;
    const double2 *L;
    int64_t ldl;
    const double2 *z;
    int64_t ldz;
    const double2 *Z;
    int64_t ldZ;
    const double2 *zR;
    int64_t ldzr;
    const double2 *ZR;
    int64_t ldZr;
    double *gs, *gv, *gm;  // outputs: n, 3n (x block, y block, z block), n
};

// Re(conj(a) * b)
__device__ inline double re_conj_mul(double2 a, double2 b) { return a.x * b.x + a.y * b.y; }

__global__ void sensitivity_kernel(SensArgs a) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (e >= a.n) return;
    double2 S = make_double2(0.0, 0.0);
    double invw = 0.0;
    if (e < a.n_vol) {
        const double w = a.vw[e];
        S = ball_integral(cbrt(3.0 * w / (4.0 * kPi)), a.k);
        invw = 1.0 / w;
    }
    double gs = 0.0, gm = 0.0, gv[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < a.nrhs; ++q) {
        const double2 p = a.P[e + q * a.ldp];
        const double2 lam = a.L[e + q * a.ldl];
        const double2 zz = a.z[e + q * a.ldz];
        const double2 zr = a.zR[e + q * a.ldzr];
        // Re p (conj zR + conj z + conj lam S / w) = Re(conj(zR + z + lam conj(S)/w) p)
        const double2 lS = cmul(lam, make_double2(S.x * invw, -S.y * invw));
        const double2 sum = make_double2(zr.x + zz.x + lS.x, zr.y + zz.y + lS.y);
        gs += re_conj_mul(sum, p);
        gm -= re_conj_mul(lam, p);
        for (int ax = 0; ax < 3; ++ax) {
            const double2 Z1 = a.Z[e + (3 * q + ax) * a.ldZ];
            const double2 Z2 = a.ZR[e + (3 * q + ax) * a.ldZr];
            gv[ax] -= re_conj_mul(make_double2(Z1.x + Z2.x, Z1.y + Z2.y), p);
        }
    }
    a.gs[e] = gs;
    a.gm[e] = gm;
    for (int ax = 0; ax < 3; ++ax) a.gv[ax * a.n + e] = gv[ax];
}

struct ChainArgs {
    DeviceMesh m;
    double k;
    const int32_t *cf_off, *cf_idx;  // cell -> adjacent faces (CSR)
    const double *gs, *gv, *gm;
    double *grad_c, *grad_rho;
};

// d(grad alpha_j along ax)/d(alpha_k) for the same-subdomain stencil of cell j.
__device__ double stencil_coef(const DeviceMesh &m, int64_t j, int ax, int64_t k) {
    const double *pc = ax == 0 ? m.px : (ax == 1 ? m.py : m.pz);
    const int dom = m.vdom[j];
    const int lo = m.vnb[6 * j + 2 * ax], hi = m.vnb[6 * j + 2 * ax + 1];
    const bool lok = lo >= 0 && m.vdom[lo] == dom;
    const bool hok = hi >= 0 && m.vdom[hi] == dom;
    if (!lok && !hok) return 0.0;
    const int64_t a = lok ? lo : j, b = hok ? hi : j;
    const double inv = 1.0 / (pc[b] - pc[a]);
    double c = 0.0;
    if (k == b) c += inv;
    if (k == a) c -= inv;
    return c;
}

__global__ void chain_kernel(ChainArgs a) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    const DeviceMesh &m = a.m;
    if (k >= m.n_vol) return;
    const double rho0 = m.rho0, c0 = m.c0;
    const double rho = m.vrho[k], c = m.vc[k], w = m.vw[k];
    const double k0 = a.k;
    const double s = w * (rho0 / rho) * k0 * k0 * ((c0 / c) * (c0 / c) - 1.0);
    const double dalpha = -rho0 / (rho * rho);       // d alpha_k / d rho_k
    // sound speed enters only through s_k
    a.grad_c[k] = a.gs[k] * (w * (rho0 / rho) * k0 * k0 * (-2.0 * c0 * c0 / (c * c * c)));
    // density: own single-layer weight and own mass function
    double g = a.gs[k] * (-s / rho) + a.gm[k] * dalpha;
    // adjacent faces: their mass function and jump weight
    for (int32_t t = a.cf_off[k]; t < a.cf_off[k + 1]; ++t) {
        const int32_t q = a.cf_idx[t];
        const int64_t f = m.n_vol + q;
        const double sgn = (m.scin[q] == k) ? 1.0 : -1.0;   // inside or outside cell
        g += a.gm[f] * (0.5 * dalpha);
        // v_f = -|face| (alpha_in - alpha_out) n_f
        const double dv = -m.sarea[q] * sgn * dalpha;
        g += dv * (a.gv[f] * m.snx[q] + a.gv[m.n + f] * m.sny[q] + a.gv[2 * m.n + f] * m.snz[q]);
    }
    // analytic density gradient: grad alpha_k = -rho0 grad(rho)_k / rho_k^2 moves
    // with rho_k by 2 rho0 grad(rho)_k / rho_k^3 (grad(rho) itself is an input)
    if (m.vgr) {
        const double rk = m.vrho[k];
        for (int ax = 0; ax < 3; ++ax)
            g += a.gv[ax * m.n + k] * m.vw[k] * (2.0 * m.rho0 * m.vgr[3 * k + ax] / (rk * rk * rk));
    }
    // grad alpha stencils that read alpha_k (own cell and same-axis neighbours)
    if (m.vnb && !m.vga && !m.vgr) {
        for (int ax = 0; ax < 3; ++ax) {
            const int64_t cand[3] = {k, m.vnb[6 * k + 2 * ax], m.vnb[6 * k + 2 * ax + 1]};
            for (int t = 0; t < 3; ++t) {
                const int64_t j = cand[t];
                if (j < 0 || m.vdom[j] != m.vdom[k]) continue;
                const double cf = stencil_coef(m, j, ax, k);
                if (cf != 0.0) g += a.gv[ax * m.n + j] * m.vw[j] * cf * dalpha;
            }
        }
    }
    a.grad_rho[k] = g;
}

__global__ void plane_wave_at_kernel(int64_t n, const double *__restrict__ tx, const double *__restrict__ ty,
                                     const double *__restrict__ tz, double k, double dx, double dy,
                                     double dz, double2 *__restrict__ b) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    double sn, cs;
    sincos(k * (tx[i] * dx + ty[i] * dy + tz[i] * dz), &sn, &cs);
    b[i] = make_double2(cs, sn);
}

}  // namespace

void launch_adjoint_rhs(const DeviceMesh &m, int f, int nrhs, const double2 *zR, int64_t ldz,
                        const double2 *ZR, int64_t ldZ, double2 *out, int64_t ldo, hipStream_t s) {
    hipLaunchKernelGGL(adjoint_rhs_kernel, dim3(blocks_for(m.n)), dim3(kT), 0, s, m.n, nrhs,
                       m.sp + static_cast<int64_t>(f) * m.n, m.vpx, m.vpy, m.vpz, zR, ldz, ZR, ldZ,
                       out, ldo);
    VSIE_HIP(hipGetLastError());
}

void launch_param_gradient(const DeviceMesh &m, const int32_t *cf_off, const int32_t *cf_idx,
                           double k, int nrhs, const double2 *P, int64_t ldp, const double2 *L,
                           int64_t ldl, const double2 *z, int64_t ldz, const double2 *Z, int64_t ldZ,
                           const double2 *zR, int64_t ldzr, const double2 *ZR, int64_t ldZr,
                           double *work, double *grad_c, double *grad_rho, hipStream_t s) {
    double *gs = work, *gm = work + m.n, *gv = work + 2 * m.n;
    SensArgs sa{m.n, m.n_vol, nrhs, k, m.vw, P, ldp, L, ldl, z, ldz, Z, ldZ, zR, ldzr, ZR, ldZr,
                gs, gv, gm};
    hipLaunchKernelGGL(sensitivity_kernel, dim3(blocks_for(m.n)), dim3(kT), 0, s, sa);
    VSIE_HIP(hipGetLastError());
    if (m.n_vol == 0) return;
    ChainArgs ca{m, k, cf_off, cf_idx, gs, gv, gm, grad_c, grad_rho};
    hipLaunchKernelGGL(chain_kernel, dim3(blocks_for(m.n_vol)), dim3(kT), 0, s, ca);
    VSIE_HIP(hipGetLastError());
}

void launch_plane_wave_at(int64_t n, const double *tx, const double *ty, const double *tz, double k,
                          double dx, double dy, double dz, double2 *b, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(plane_wave_at_kernel, dim3(blocks_for(n)), dim3(kT), 0, s, n, tx, ty, tz, k,
                       dx, dy, dz, b);
    VSIE_HIP(hipGetLastError());
}

}  // namespace vsie
