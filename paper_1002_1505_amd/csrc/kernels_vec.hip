// Vector kernels of the DDA solver on gfx950: incident field, BiCGstab
// updates with fused FP64 inner-product partials, per-right-hand-side scalar
// updates, precision conversion for the FP64 refinement, layout conversion at
// the ABI boundary, cross-section and scattering-amplitude reductions.
//
// Vectors are [rhs][3][Npad] complex; a grid is (blocks per rhs, nrhs), every
// thread handles VPT consecutive-by-stride elements.  Inner products are
// accumulated in FP64: per-thread, wavefront shuffle, LDS, then a per-rhs
// second stage over the block partials.
#include "dda_internal.h"

#define HIP_TRY(x)                       \
    do {                                 \
        hipError_t e_ = (x);             \
        if (e_ != hipSuccess) return e_; \
    } while (0)

namespace {
constexpr int VT = 256;  // threads per vector block
constexpr int VPT = 4;   // elements per thread
constexpr int VB = VT * VPT;

__device__ __forceinline__ bool inactive(const int* active, int rhs) { return active && !active[rhs]; }

template <class T>
__device__ __forceinline__ void acc_dot(double2& a, Cx<T> u, Cx<T> v) {
    // conj(u) * v in FP64
    const double ur = u.re, ui = u.im, vr = v.re, vi = v.im;
    a.x += ur * vr + ui * vi;
    a.y += ur * vi - ui * vr;
}

// Block reduction of up to 4 complex partial sums; thread 0 writes
// partials[rhs][slot][blockIdx.x].
__device__ void store_partials(const double2* a, int nslot, double* partials, int rhs, int nblk) {
    __shared__ double sh[16];
    for (int s = 0; s < nslot; ++s) {
        const double re = block_sum(a[s].x, sh);
        const double im = block_sum(a[s].y, sh);
        if (threadIdx.x == 0) {
            double* o = partials + (((size_t)rhs * 4 + s) * nblk + blockIdx.x) * 2;
            o[0] = re;
            o[1] = im;
        }
    }
}

template <class T>
__global__ void __launch_bounds__(VT) k_einc(Geo g, double ox, double oy, double oz, const WaveDev* __restrict__ w,
                                             Cx<T>* __restrict__ E) {
    const int rhs = blockIdx.y;
    const WaveDev wv = w[rhs];
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < g.Npad; j += gridDim.x * blockDim.x) {
        Cx<T> o[3] = {{0, 0}, {0, 0}, {0, 0}};
        if (j < g.N) {
            const uint32_t s = g.site_xyz[j];
            const double x = (double)(s & 1023) - ox, y = (double)((s >> 10) & 1023) - oy,
                         z = (double)(s >> 20) - oz;
            double sn, cs;
            sincos(wv.k * (wv.khat[0] * x + wv.khat[1] * y + wv.khat[2] * z), &sn, &cs);
            for (int c = 0; c < 3; ++c) {
                const double er = wv.e[2 * c], ei = wv.e[2 * c + 1];
                o[c] = Cx<T>{(T)(er * cs - ei * sn), (T)(er * sn + ei * cs)};
            }
        }
        for (int c = 0; c < 3; ++c) E[((size_t)rhs * 3 + c) * g.Npad + j] = o[c];
    }
}

template <class T>
__global__ void k_fillv(Cx<T>* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = Cx<T>{0, 0};
}
__global__ void k_filli(int* p, int v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// p = r + beta (p - omega v); on restart rhat = r, p = r.
template <class T>
__global__ void __launch_bounds__(VT) k_bicg_p(int V, Cx<T>* __restrict__ p, const Cx<T>* __restrict__ r,
                                               const Cx<T>* __restrict__ v, Cx<T>* __restrict__ rhat,
                                               const BiState* __restrict__ st, const int* __restrict__ active) {
    const int rhs = blockIdx.y;
    if (inactive(active, rhs)) return;
    const BiState s = st[rhs];
    const size_t o = (size_t)rhs * V;
    const Cx<T> beta = {(T)s.beta[0], (T)s.beta[1]}, omega = {(T)s.omega[0], (T)s.omega[1]};
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i < V) {
            const Cx<T> ri = r[o + i];
            if (s.restart) {
                rhat[o + i] = ri;
                p[o + i] = ri;
            } else {
                p[o + i] = ri + beta * (p[o + i] - omega * v[o + i]);
            }
        }
    }
}

// partials[rhs][0..npair) = sum conj(a_k) b_k
template <class T>
__global__ void __launch_bounds__(VT) k_dot(int V, int npair, const Cx<T>* __restrict__ a0,
                                            const Cx<T>* __restrict__ b0, const Cx<T>* __restrict__ a1,
                                            const Cx<T>* __restrict__ b1, double* __restrict__ partials,
                                            const int* __restrict__ active) {
    const int rhs = blockIdx.y;
    if (inactive(active, rhs)) return;
    const size_t o = (size_t)rhs * V;
    double2 acc[2] = {{0, 0}, {0, 0}};
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i < V) {
            acc_dot(acc[0], a0[o + i], b0[o + i]);
            if (npair > 1) acc_dot(acc[1], a1[o + i], b1[o + i]);
        }
    }
    store_partials(acc, npair, partials, rhs, gridDim.x);
}

// s = r - alpha v
template <class T>
__global__ void __launch_bounds__(VT) k_bicg_s(int V, Cx<T>* __restrict__ s, const Cx<T>* __restrict__ r,
                                               const Cx<T>* __restrict__ v, const BiState* __restrict__ st,
                                               const int* __restrict__ active) {
    const int rhs = blockIdx.y;
    if (inactive(active, rhs)) return;
    const size_t o = (size_t)rhs * V;
    const Cx<T> alpha = {(T)st[rhs].alpha[0], (T)st[rhs].alpha[1]};
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i < V) s[o + i] = r[o + i] - alpha * v[o + i];
    }
}

// x += alpha p + omega s; r = s - omega t; partials <rhat, r>, <r, r>
template <class T>
__global__ void __launch_bounds__(VT) k_bicg_xr(int V, Cx<T>* __restrict__ x, Cx<T>* __restrict__ r,
                                                const Cx<T>* __restrict__ p, const Cx<T>* __restrict__ s,
                                                const Cx<T>* __restrict__ t, const Cx<T>* __restrict__ rhat,
                                                const BiState* __restrict__ st, double* __restrict__ partials,
                                                const int* __restrict__ active) {
    const int rhs = blockIdx.y;
    if (inactive(active, rhs)) return;
    const size_t o = (size_t)rhs * V;
    const Cx<T> alpha = {(T)st[rhs].alpha[0], (T)st[rhs].alpha[1]};
    const Cx<T> omega = {(T)st[rhs].omega[0], (T)st[rhs].omega[1]};
    double2 acc[2] = {{0, 0}, {0, 0}};
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i < V) {
            const Cx<T> si = s[o + i];
            x[o + i] = x[o + i] + alpha * p[o + i] + omega * si;
            const Cx<T> ri = si - omega * t[o + i];
            r[o + i] = ri;
            acc_dot(acc[0], rhat[o + i], ri);
            acc_dot(acc[1], ri, ri);
        }
    }
    store_partials(acc, 2, partials, rhs, gridDim.x);
}

__device__ __forceinline__ double2 reduce_slot(const double* partials, int rhs, int slot, int nblk, double* sh) {
    double re = 0, im = 0;
    const double* p = partials + ((size_t)rhs * 4 + slot) * nblk * 2;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        re += p[2 * i];
        im += p[2 * i + 1];
    }
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    return make_double2(re, im);
}

// One block per rhs.
//  which 0: alpha = rho / <rhat, v>       (partials slot 0); breakdown -> alpha = 0, restart
//           (in the fused iteration the forward pass of s forms alpha itself)
//  which 1: omega = <t, s> / <t, t>       (slots 0, 1); breakdown -> omega = 0, restart
//  which 2: rho' = <rhat, r>, rr = <r, r> (slots 0, 1); beta, convergence, iteration count
//  which 3: the fused end of an iteration that never forms r = s - omega t:
//           omega from <t, s>, <t, t> (slots 0, 1.re), then
//           rho' = <rhat, s> - omega <rhat, t> (slots 2, 3) and
//           rr = ||s||^2 - 2 Re(conj(omega) <t, s>) + |omega|^2 ||t||^2 (slot 1.im),
//           followed by the which-2 logic; marks the x, r update pending with
//           the direction in buffer kpar
__device__ void finish_iteration(BiState& s, double2 a, double2 b, int* active, int rhs) {
    // a = <rhat, r>, b.x = <r, r>
    const double2 rho = make_double2(s.rho[0], s.rho[1]);
    s.it += 1;
    s.rr = b.x;
    if (s.trace && s.it <= s.tcap) s.trace[s.it - 1] = b.x;
    if (s.frs > 0 && s.it % s.frs == 0) s.restart = 1;
    const double2 al = make_double2(s.alpha[0], s.alpha[1]), om = make_double2(s.omega[0], s.omega[1]);
    const double rn = sqrt(a.x * a.x + a.y * a.y);
    if (s.restart || !(rn > 1e-14 * b.x) || (om.x == 0 && om.y == 0)) {
        s.restart = 1;
        s.rho[0] = b.x;
        s.rho[1] = 0;
    } else {
        const double2 be = cmul2(cdiv(a, rho), cdiv(al, om));
        s.beta[0] = be.x;
        s.beta[1] = be.y;
        s.rho[0] = a.x;
        s.rho[1] = a.y;
    }
    if (!(b.x > s.tol2)) s.conv = 1;
    if (s.conv || s.it >= s.maxit || !isfinite(b.x)) active[rhs] = 0;
}

constexpr int SCALAR_THREADS = 1024;

__global__ void __launch_bounds__(SCALAR_THREADS)
    k_scalars(int which, int nblk, BiState* __restrict__ st, const double* __restrict__ partials,
              int* __restrict__ active, int kpar) {
    __shared__ double sh[8 * (SCALAR_THREADS / 64)];
    const int rhs = blockIdx.x;
    if (!active[rhs]) return;
    // all slots the step needs in one pass over the block partials: the
    // loads of every slot are issued together (one memory round trip per
    // SCALAR_THREADS partials instead of one per slot and stride)
    const int nslot = which == 0 ? 1 : (which == 3 ? 4 : 2);
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double2* p2 = reinterpret_cast<const double2*>(partials) + (size_t)rhs * 4 * nblk;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        double2 e[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) e[q] = q < nslot ? p2[(size_t)q * nblk + i] : make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[2 * q] += e[q].x;
            v[2 * q + 1] += e[q].y;
        }
    }
    block_sum_n<8>(v, sh);
    if (threadIdx.x != 0) return;
    const double2 a = make_double2(v[0], v[1]), b = make_double2(v[2], v[3]);
    const double2 c2 = make_double2(v[4], v[5]), d2 = make_double2(v[6], v[7]);
    BiState s = st[rhs];
    if (which == 3) {
        // a = <t, s>, b = (<t, t>, <s, s>), c2 = <rhat, s>, d2 = <rhat, t>
        double2 om = make_double2(0, 0);
        if (!(b.x > 0)) {
            s.restart = 1;
        } else {
            om = make_double2(a.x / b.x, a.y / b.x);
            if (om.x == 0 && om.y == 0) s.restart = 1;
        }
        s.omega[0] = om.x;
        s.omega[1] = om.y;
        const double2 rho2 = make_double2(c2.x - (om.x * d2.x - om.y * d2.y), c2.y - (om.x * d2.y + om.y * d2.x));
        const double rr = fmax(0.0, b.y - 2.0 * (om.x * a.x + om.y * a.y) + (om.x * om.x + om.y * om.y) * b.x);
        finish_iteration(s, rho2, make_double2(rr, 0), active, rhs);
        s.pend = 1;
        s.pbuf = kpar;
        st[rhs] = s;
        return;
    }
    const double2 rho = make_double2(s.rho[0], s.rho[1]);
    if (which == 0) {
        s.restart = 0;
        const double an = sqrt(a.x * a.x + a.y * a.y);
        if (!(an > 1e-300) || !(an > 1e-14 * s.rr)) {
            s.alpha[0] = s.alpha[1] = 0;
            s.restart = 1;
        } else {
            const double2 al = cdiv(rho, a);
            s.alpha[0] = al.x;
            s.alpha[1] = al.y;
        }
    } else if (which == 1) {
        // a = <t, s>, b = <t, t>
        if (!(b.x > 0)) {
            s.omega[0] = s.omega[1] = 0;
            s.restart = 1;
        } else {
            s.omega[0] = a.x / b.x;
            s.omega[1] = a.y / b.x;
            if (s.omega[0] == 0 && s.omega[1] == 0) s.restart = 1;
        }
    } else {
        (void)rho;
        finish_iteration(s, a, b, active, rhs);
    }
    st[rhs] = s;
}

// ---------------------------------------------------------------------------
// BiCGstab(2): per-rhs scalar steps and the vector updates of a cycle.
// ---------------------------------------------------------------------------
__global__ void k_l2_state_init(int nblk, BiState* __restrict__ st, const double* __restrict__ partials,
                                const double* __restrict__ tol_rel2, const int* __restrict__ maxit,
                                int* __restrict__ active, int frs, double* trace, int tcap) {
    __shared__ double sh[16];
    const int rhs = blockIdx.x;
    const double2 a = reduce_slot(partials, rhs, 0, nblk, sh);
    if (threadIdx.x != 0) return;
    BiState s;
    s.rho[0] = 1;
    s.rho[1] = 0;
    s.alpha[0] = s.alpha[1] = 0;
    s.omega[0] = 1;
    s.omega[1] = 0;
    s.beta[0] = s.beta[1] = 0;
    s.rr = a.x;
    s.tol2 = tol_rel2[rhs] * a.x;
    s.it = 0;
    s.maxit = maxit[rhs];
    s.restart = 0;
    s.conv = (a.x <= s.tol2) ? 1 : 0;
    s.pend = 0;
    s.pbuf = 0;
    s.frs = frs;
    s.tcap = trace ? tcap : 0;
    s.trace = trace ? trace + (size_t)rhs * tcap : nullptr;
    s.ex[0] = a.x;  // <rt, r0> with rt = r0
    s.ex[1] = 0;
    s.ex[2] = s.ex[3] = s.ex[4] = s.ex[5] = 0;
    st[rhs] = s;
    active[rhs] = (maxit[rhs] > 0 && !s.conv && a.x > 0) ? 1 : 0;
    if (a.x == 0) st[rhs].conv = 1;
}

__global__ void __launch_bounds__(SCALAR_THREADS)
    k_l2_scalars(int which, int nblk, BiState* __restrict__ st, const double* __restrict__ partials,
                 int* __restrict__ active) {
    __shared__ double sh[8 * (SCALAR_THREADS / 64)];
    const int rhs = blockIdx.x;
    if (!active[rhs]) return;
    const int nslot = (which == 3) ? 4 : (which == 4 ? 2 : (which == 0 ? 0 : 1));
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double2* p2 = reinterpret_cast<const double2*>(partials) + (size_t)rhs * 4 * nblk;
    for (int i = threadIdx.x; i < nblk && nslot > 0; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q < nslot) {
                const double2 e = p2[(size_t)q * nblk + i];
                v[2 * q] += e.x;
                v[2 * q + 1] += e.y;
            }
        }
    }
    block_sum_n<8>(v, sh);
    if (threadIdx.x != 0) return;
    BiState s = st[rhs];
    const double2 a = make_double2(v[0], v[1]);
    const double tiny = 1e-14 * s.rr;
    if (which == 0) {
        // cycle start: rho0 = -omega rho0, beta = alpha rho1 / rho0, rho0 = rho1;
        // a restart (breakdown or forced) starts over with rt = r0: beta = 0
        double2 rho1 = make_double2(s.ex[0], s.ex[1]);
        const double2 r0n = cmul2(make_double2(-s.omega[0], -s.omega[1]), make_double2(s.rho[0], s.rho[1]));
        const double an = sqrt(r0n.x * r0n.x + r0n.y * r0n.y);
        if (s.pend || !(an > 1e-300) || !(an > 1e-14 * s.rr)) {
            s.restart = 1;
            s.pend = 0;
            rho1 = make_double2(s.rr, 0.0);
            s.beta[0] = s.beta[1] = 0;
            s.alpha[0] = s.alpha[1] = 0;
        } else {
            const double2 be = cmul2(make_double2(s.alpha[0], s.alpha[1]), cdiv(rho1, r0n));
            s.beta[0] = be.x;
            s.beta[1] = be.y;
        }
        s.rho[0] = rho1.x;
        s.rho[1] = rho1.y;
    } else if (which == 1) {
        // alpha = rho0 / <rt, u_{j+1}>; a vanishing denominator leaves x and r
        // as they are (alpha = 0) and restarts at the next cycle
        s.restart = 0;
        const double an = sqrt(a.x * a.x + a.y * a.y);
        if (!(an > 1e-300) || !(an > tiny)) {
            s.alpha[0] = s.alpha[1] = 0;
            s.pend = 1;
        } else {
            const double2 al = cdiv(make_double2(s.rho[0], s.rho[1]), a);
            s.alpha[0] = al.x;
            s.alpha[1] = al.y;
        }
    } else if (which == 2) {
        // second BiCG step: rho1 = <rt, r1>, beta = alpha rho1 / rho0, rho0 = rho1
        const double2 rho0 = make_double2(s.rho[0], s.rho[1]);
        const double rn = sqrt(rho0.x * rho0.x + rho0.y * rho0.y);
        if (!(rn > 1e-300) || !(rn > tiny)) {
            s.beta[0] = s.beta[1] = 0;
            s.pend = 1;
        } else {
            const double2 be = cmul2(make_double2(s.alpha[0], s.alpha[1]), cdiv(a, rho0));
            s.beta[0] = be.x;
            s.beta[1] = be.y;
        }
        s.rho[0] = a.x;
        s.rho[1] = a.y;
    } else if (which == 3) {
        // MR step over r1, r2: Gram-Schmidt r2' = r2 - tau r1, then
        // gamma'_1 = <r1, r0> / sigma1, gamma'_2 = <r2', r0> / sigma2,
        // gamma_2 = gamma'_2 = omega, gamma_1 = gamma'_1 - tau gamma_2
        const double2 b = make_double2(v[4], v[5]), d = make_double2(v[6], v[7]);
        const double s1 = v[3], n22 = v[2];
        double2 g1 = make_double2(0, 0), g2 = make_double2(0, 0);
        if (s1 > 1e-300) {
            const double2 tau = make_double2(a.x / s1, -a.y / s1);  // <r1, r2> / sigma1
            const double s2 = n22 - (a.x * a.x + a.y * a.y) / s1;
            const double2 gp1 = make_double2(b.x / s1, -b.y / s1);   // <r1, r0> / sigma1
            if (s2 > 1e-14 * n22 && s2 > 1e-300) {
                // <r2', r0> = <r2, r0> - conj(tau) <r1, r0> = conj(d) - (a / sigma1) conj(b)
                const double2 ab = cmul2(make_double2(a.x / s1, a.y / s1), make_double2(b.x, -b.y));
                const double2 q = make_double2(d.x - ab.x, -d.y - ab.y);
                g2 = make_double2(q.x / s2, q.y / s2);
                const double2 tg = cmul2(tau, g2);
                g1 = make_double2(gp1.x - tg.x, gp1.y - tg.y);
            } else {
                g1 = gp1;  // r2 adds nothing beyond r1: degree-one polynomial
            }
        }
        if (g2.x == 0 && g2.y == 0) s.pend = 1;  // omega = 0: no BiCG recurrence after this cycle
        s.omega[0] = g2.x;
        s.omega[1] = g2.y;
        s.ex[2] = g1.x;
        s.ex[3] = g1.y;
        s.ex[4] = g2.x;
        s.ex[5] = g2.y;
    } else {
        // cycle end: ||r0||^2 (slot 1), <rt, r0> for the next cycle (slot 0)
        const double rr = v[2];
        s.it += 2;
        s.rr = rr;
        if (s.trace) {
            if (s.it - 1 <= s.tcap) s.trace[s.it - 2] = rr;
            if (s.it <= s.tcap) s.trace[s.it - 1] = rr;
        }
        s.ex[0] = a.x;
        s.ex[1] = a.y;
        if (s.frs > 0 && s.it % s.frs == 0) s.pend = 1;
        if (!(rr > s.tol2)) s.conv = 1;
        if (s.conv || s.it >= s.maxit || !isfinite(rr)) active[rhs] = 0;
    }
    st[rhs] = s;
}

template <class T>
__global__ void __launch_bounds__(VT) k_l2_update(int step, int V, Cx<T>* __restrict__ x, Cx<T>* __restrict__ r0,
                                                  Cx<T>* __restrict__ rt, Cx<T>* __restrict__ u0,
                                                  Cx<T>* __restrict__ u1, const Cx<T>* __restrict__ u2,
                                                  Cx<T>* __restrict__ r1, const Cx<T>* __restrict__ r2,
                                                  const BiState* __restrict__ st, double* __restrict__ partials,
                                                  const int* __restrict__ active) {
    const int rhs = blockIdx.y;
    if (inactive(active, rhs)) return;
    const BiState b = st[rhs];
    const Cx<T> al = {(T)b.alpha[0], (T)b.alpha[1]}, be = {(T)b.beta[0], (T)b.beta[1]};
    const Cx<T> g1 = {(T)b.ex[2], (T)b.ex[3]}, g2 = {(T)b.ex[4], (T)b.ex[5]};
    const size_t o = (size_t)rhs * V;
    double2 acc[2] = {{0, 0}, {0, 0}};
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i >= V) continue;
        const size_t e = o + i;
        if (step == 1) {
            const Cx<T> r = r0[e];
            u0[e] = r - be * u0[e];
            if (b.restart) rt[e] = r;
        } else if (step == 2) {
            r0[e] = r0[e] - al * u1[e];
            x[e] = x[e] + al * u0[e];
        } else if (step == 3) {
            u0[e] = r0[e] - be * u0[e];
            u1[e] = r1[e] - be * u1[e];
        } else if (step == 4) {
            const Cx<T> a1 = u1[e];
            r0[e] = r0[e] - al * a1;
            r1[e] = r1[e] - al * u2[e];
            x[e] = x[e] + al * u0[e];
        } else {
            const Cx<T> q0 = r0[e], q1 = r1[e];
            x[e] = x[e] + g1 * q0 + g2 * q1;
            const Cx<T> rn = q0 - g1 * q1 - g2 * r2[e];
            r0[e] = rn;
            u0[e] = u0[e] - g1 * u1[e] - g2 * u2[e];
            acc_dot(acc[0], rt[e], rn);
            acc_dot(acc[1], rn, rn);
        }
    }
    if (step == 5) store_partials(acc, 2, partials, rhs, gridDim.x);
}

// slot 0 <r2, r1>, slot 1 (||r2||^2, ||r1||^2), slot 2 <r0, r1>, slot 3 <r0, r2>
template <class T>
__global__ void __launch_bounds__(VT) k_l2_mrdot(int V, const Cx<T>* __restrict__ r0, const Cx<T>* __restrict__ r1,
                                                 const Cx<T>* __restrict__ r2, double* __restrict__ partials,
                                                 const int* __restrict__ active) {
    const int rhs = blockIdx.y;
    if (inactive(active, rhs)) return;
    const size_t o = (size_t)rhs * V;
    double2 acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i >= V) continue;
        const Cx<T> a0 = r0[o + i], a1 = r1[o + i], a2 = r2[o + i];
        acc_dot(acc[0], a2, a1);
        const double n2 = (double)a2.re * a2.re + (double)a2.im * a2.im;
        const double n1 = (double)a1.re * a1.re + (double)a1.im * a1.im;
        acc[1].x += n2;
        acc[1].y += n1;
        acc_dot(acc[2], a0, a1);
        acc_dot(acc[3], a0, a2);
    }
    store_partials(acc, 4, partials, rhs, gridDim.x);
}

// ---------------------------------------------------------------------------
// Anisotropic compositions: the tensor part of the diagonal term and of the
// absorption sum.  tens: [rhs][ncomp][6] complex (xx, xy, xz, yy, yz, zz) of
// the symmetric 3 x 3 1/alpha, zero for isotropic compositions (whose
// scalar 1/alpha the matvec passes apply).
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_aniso_diag(Geo g, const Cx<T>* __restrict__ x, Cx<T>* __restrict__ y,
                                                    const Cx<T>* __restrict__ tens, T sgn) {
    const int rhs = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.N) return;
    const Cx<T>* tc = tens + ((size_t)rhs * g.ncomp + g.site_comp[j]) * 6;
    const Cx<T> t[6] = {tc[0], tc[1], tc[2], tc[3], tc[4], tc[5]};
    bool any = false;
#pragma unroll
    for (int q = 0; q < 6; ++q) any |= (t[q].re != 0 || t[q].im != 0);
    if (!any) return;
    const size_t o = (size_t)rhs * 3 * g.Npad + j;
    const Cx<T> x0 = x[o], x1 = x[o + g.Npad], x2 = x[o + 2 * (size_t)g.Npad];
    y[o] = y[o] + sgn * (t[0] * x0 + t[1] * x1 + t[2] * x2);
    y[o + g.Npad] = y[o + g.Npad] + sgn * (t[1] * x0 + t[3] * x1 + t[4] * x2);
    y[o + 2 * (size_t)g.Npad] = y[o + 2 * (size_t)g.Npad] + sgn * (t[2] * x0 + t[4] * x1 + t[5] * x2);
}

// partials slot 0 (re): sum over anisotropic sites of Im(P . conj(T) P^*) = -Im(P^H T P)
__global__ void __launch_bounds__(VT) k_aniso_abs(Geo g, const Cx<double>* __restrict__ P,
                                                  const Cx<double>* __restrict__ tens, double* __restrict__ partials) {
    const int rhs = blockIdx.y;
    double2 acc[1] = {{0, 0}};
    for (int j = blockIdx.x * VT + threadIdx.x; j < g.N; j += gridDim.x * VT) {
        const Cx<double>* tc = tens + ((size_t)rhs * g.ncomp + g.site_comp[j]) * 6;
        const size_t o = (size_t)rhs * 3 * g.Npad + j;
        const Cx<double> p[3] = {P[o], P[o + g.Npad], P[o + 2 * (size_t)g.Npad]};
        const int ix[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
        double im = 0;
        for (int a = 0; a < 3; ++a) {
            Cx<double> tp = {0, 0};
            for (int b = 0; b < 3; ++b) tp = tp + tc[ix[a][b]] * p[b];
            im += p[a].re * tp.im - p[a].im * tp.re;  // Im(conj(p_a) (T p)_a)
        }
        acc[0].x -= im;
    }
    store_partials(acc, 1, partials, rhs, gridDim.x);
}

// Pending x, r update of a fused iteration.
template <class T>
__global__ void __launch_bounds__(VT) k_bicg_flush(int V, Cx<T>* __restrict__ x, Cx<T>* __restrict__ r,
                                                   const Cx<T>* __restrict__ p0, const Cx<T>* __restrict__ p1,
                                                   const Cx<T>* __restrict__ s, const Cx<T>* __restrict__ t,
                                                   const BiState* __restrict__ st) {
    const int rhs = blockIdx.y;
    const BiState b = st[rhs];
    // an iteration that ended non-finite is not applied
    if (!b.pend || !isfinite(b.rr)) return;
    const Cx<T> al = {(T)b.alpha[0], (T)b.alpha[1]}, om = {(T)b.omega[0], (T)b.omega[1]};
    const Cx<T>* p = b.pbuf ? p1 : p0;
    const size_t o = (size_t)rhs * V;
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i < V) {
            const Cx<T> si = s[o + i];
            x[o + i] = x[o + i] + al * p[o + i] + om * si;
            r[o + i] = si - om * t[o + i];
        }
    }
}

// Direction update of a fused iteration, ahead of its forward pass: first the
// pending x, r update of the previous iteration when st.pend (x += alpha p +
// omega s, r = s - omega t), then p' = r + beta (p - omega v), or p' = r and
// rhat = r on restart.  p' goes to its own buffer (pout never aliases p).
template <class T>
__global__ void __launch_bounds__(VT) k_bicg_upd(int V, Cx<T>* __restrict__ x, Cx<T>* __restrict__ r,
                                                 const Cx<T>* __restrict__ p, Cx<T>* __restrict__ pout,
                                                 const Cx<T>* __restrict__ v, Cx<T>* __restrict__ rhat,
                                                 const Cx<T>* __restrict__ s, const Cx<T>* __restrict__ t,
                                                 const BiState* __restrict__ st, const int* __restrict__ active) {
    const int rhs = blockIdx.y;
    if (inactive(active, rhs)) return;
    const BiState b = st[rhs];
    const Cx<T> al = {(T)b.alpha[0], (T)b.alpha[1]}, om = {(T)b.omega[0], (T)b.omega[1]};
    const Cx<T> be = {(T)b.beta[0], (T)b.beta[1]};
    const size_t o = (size_t)rhs * V;
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i < V) {
            const Cx<T> pi = p[o + i];
            Cx<T> ri;
            if (b.pend) {
                const Cx<T> si = s[o + i];
                ri = si - om * t[o + i];
                r[o + i] = ri;
                x[o + i] = x[o + i] + al * pi + om * si;
            } else {
                ri = r[o + i];
            }
            if (b.restart) {
                rhat[o + i] = ri;
                pout[o + i] = ri;
            } else {
                pout[o + i] = ri + be * (pi - om * v[o + i]);
            }
        }
    }
}

__global__ void k_clear_pend(BiState* st, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) st[i].pend = 0;
}

// State initialisation from <r, r> in slot 0.
__global__ void k_state_init(int nblk, BiState* __restrict__ st, const double* __restrict__ partials,
                             const double* __restrict__ tol_rel2, const int* __restrict__ maxit,
                             int* __restrict__ active, int frs, double* trace, int tcap) {
    __shared__ double sh[16];
    const int rhs = blockIdx.x;
    const double2 a = reduce_slot(partials, rhs, 0, nblk, sh);
    if (threadIdx.x != 0) return;
    BiState s;
    s.rho[0] = a.x;
    s.rho[1] = 0;
    s.alpha[0] = s.alpha[1] = 0;
    s.omega[0] = 1;
    s.omega[1] = 0;
    s.beta[0] = s.beta[1] = 0;
    s.rr = a.x;
    s.tol2 = tol_rel2[rhs] * a.x;
    s.it = 0;
    s.maxit = maxit[rhs];
    s.restart = 1;
    s.conv = (a.x <= s.tol2) ? 1 : 0;
    s.pend = 0;
    s.pbuf = 0;
    s.frs = frs;
    s.tcap = trace ? tcap : 0;
    s.trace = trace ? trace + (size_t)rhs * tcap : nullptr;
    st[rhs] = s;
    active[rhs] = (maxit[rhs] > 0 && !s.conv && a.x > 0) ? 1 : 0;
    if (a.x == 0) st[rhs].conv = 1;
}

// x = 0, r = rhat = p = b, v = 0
template <class T>
__global__ void __launch_bounds__(VT) k_bicg_init(int V, const Cx<T>* __restrict__ b, Cx<T>* __restrict__ x,
                                                  Cx<T>* __restrict__ r, Cx<T>* __restrict__ rhat,
                                                  Cx<T>* __restrict__ p, Cx<T>* __restrict__ v) {
    const size_t o = (size_t)blockIdx.y * V;
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i < V) {
            const Cx<T> bi = b[o + i];
            x[o + i] = Cx<T>{0, 0};
            r[o + i] = bi;
            rhat[o + i] = bi;
            p[o + i] = bi;
            v[o + i] = Cx<T>{0, 0};
        }
    }
}

__global__ void __launch_bounds__(VT) k_demote(int V, const Cx<double>* __restrict__ r64, Cx<float>* __restrict__ r32,
                                               const double* __restrict__ scale, const int* __restrict__ mask) {
    const int rhs = blockIdx.y;
    if (inactive(mask, rhs)) return;
    const size_t o = (size_t)rhs * V;
    const double sc = scale[rhs];
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i < V) {
            const Cx<double> a = r64[o + i];
            r32[o + i] = Cx<float>{(float)(a.re * sc), (float)(a.im * sc)};
        }
    }
}

__global__ void __launch_bounds__(VT) k_promote_add(int V, Cx<double>* __restrict__ x64,
                                                    const Cx<float>* __restrict__ d32, const double* __restrict__ scale,
                                                    const int* __restrict__ mask, const BiState* __restrict__ st) {
    const int rhs = blockIdx.y;
    if (inactive(mask, rhs) || !isfinite(st[rhs].rr)) return;
    const size_t o = (size_t)rhs * V;
    const double sc = 1.0 / scale[rhs];
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i < V) {
            const Cx<float> d = d32[o + i];
            x64[o + i] = x64[o + i] + Cx<double>{sc * (double)d.re, sc * (double)d.im};
        }
    }
}

template <class T>
__global__ void __launch_bounds__(VT) k_axpy_masked(int V, Cx<T>* __restrict__ x, const Cx<T>* __restrict__ d,
                                                    const int* __restrict__ mask, const BiState* __restrict__ st) {
    const int rhs = blockIdx.y;
    if (inactive(mask, rhs) || !isfinite(st[rhs].rr)) return;
    const size_t o = (size_t)rhs * V;
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i < V) x[o + i] = x[o + i] + d[o + i];
    }
}

template <class T>
__global__ void __launch_bounds__(VT) k_norm2_part(int V, const Cx<T>* __restrict__ v, double* __restrict__ partials) {
    const int rhs = blockIdx.y;
    const size_t o = (size_t)rhs * V;
    double2 acc[1] = {{0, 0}};
    for (int k = 0; k < VPT; ++k) {
        const int i = blockIdx.x * VB + k * VT + threadIdx.x;
        if (i < V) acc_dot(acc[0], v[o + i], v[o + i]);
    }
    store_partials(acc, 1, partials, rhs, gridDim.x);
}

__global__ void k_norm2_final(int nblk, const double* __restrict__ partials, double* __restrict__ out) {
    __shared__ double sh[16];
    const double2 a = reduce_slot(partials, blockIdx.x, 0, nblk, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = a.x;
}

template <class T>
__global__ void k_from_abi(int N, int Npad, const int* __restrict__ perm, const Cx<double>* __restrict__ in,
                           Cx<T>* __restrict__ out) {
    const int rhs = blockIdx.y;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < Npad; j += gridDim.x * blockDim.x) {
        const int ja = j < N ? perm[j] : 0;
        for (int c = 0; c < 3; ++c) {
            Cx<T> v = {0, 0};
            if (j < N) {
                const Cx<double> a = in[((size_t)rhs * N + ja) * 3 + c];
                v = Cx<T>{(T)a.re, (T)a.im};
            }
            out[((size_t)rhs * 3 + c) * Npad + j] = v;
        }
    }
}

template <class T>
__global__ void k_to_abi(int N, int Npad, const int* __restrict__ perm, const Cx<T>* __restrict__ in,
                         Cx<double>* __restrict__ out) {
    const int rhs = blockIdx.y;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
        const int ja = perm[j];
        for (int c = 0; c < 3; ++c) {
            const Cx<T> a = in[((size_t)rhs * 3 + c) * Npad + j];
            out[((size_t)rhs * N + ja) * 3 + c] = Cx<double>{(double)a.re, (double)a.im};
        }
    }
}

// partials slots: 0 = (sum Im(E^*.P), 0), 1 = (sum |P|^2 (-Im ainv - 2/3 k^3), 0)
__global__ void __launch_bounds__(VT) k_xsec_part(Geo g, const Cx<double>* __restrict__ E,
                                                  const Cx<double>* __restrict__ P,
                                                  const Cx<double>* __restrict__ ainv, double k3,
                                                  double* __restrict__ partials) {
    const int rhs = blockIdx.y;
    double2 acc[2] = {{0, 0}, {0, 0}};
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < g.N; j += gridDim.x * blockDim.x) {
        double p2 = 0;
        for (int c = 0; c < 3; ++c) {
            const size_t i = ((size_t)rhs * 3 + c) * g.Npad + j;
            const Cx<double> e = E[i], p = P[i];
            acc[0].x += e.re * p.im - e.im * p.re;  // Im(conj(e) p)
            acc[0].y += e.re * p.re + e.im * p.im;  // Re(conj(e) p)
            p2 += p.re * p.re + p.im * p.im;
        }
        const Cx<double> ai = ainv[(size_t)rhs * g.ncomp + g.site_comp[j]];
        acc[1].x += p2 * (-ai.im - (2.0 / 3.0) * k3);
    }
    store_partials(acc, 2, partials, rhs, gridDim.x);
}

__global__ void k_xsec_final(int nblk, const double* __restrict__ partials, double* __restrict__ out) {
    __shared__ double sh[16];
    const double2 a = reduce_slot(partials, blockIdx.x, 0, nblk, sh);
    const double2 b = reduce_slot(partials, blockIdx.x, 1, nblk, sh);
    if (threadIdx.x == 0) {
        out[3 * blockIdx.x] = a.x;
        out[3 * blockIdx.x + 1] = b.x;
        out[3 * blockIdx.x + 2] = a.y;
    }
}

// Pair sums for the cross sections of linear combinations of two solutions
// (slots s0, s1 of one group): S_ab = sum_j conj(E_a,j) . P_b,j and
// G_ab = sum_j w_j conj(P_a,j) . P_b,j with w_j = -Im(1/alpha_j) - (2/3) k^3
// (1/alpha of slot s0).  Block partials, (re, im) of S00 S01 S10 S11 G00 G01
// G10 G11: part[((pair * gridDim.x) + blk) * 16 + q].
__global__ void __launch_bounds__(256) k_xsec_pair(Geo g, const Cx<double>* __restrict__ E,
                                                   const Cx<double>* __restrict__ P,
                                                   const Cx<double>* __restrict__ ainv, double k3,
                                                   const int* __restrict__ slots, double* __restrict__ part) {
    __shared__ double sh[16 * 4];
    const int pr = blockIdx.y;
    const int s0 = slots[2 * pr], s1 = slots[2 * pr + 1];
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < g.N; j += gridDim.x * blockDim.x) {
        const double w = -ainv[(size_t)s0 * g.ncomp + g.site_comp[j]].im - (2.0 / 3.0) * k3;
        for (int c = 0; c < 3; ++c) {
            const Cx<double> e[2] = {E[((size_t)s0 * 3 + c) * g.Npad + j], E[((size_t)s1 * 3 + c) * g.Npad + j]};
            const Cx<double> p[2] = {P[((size_t)s0 * 3 + c) * g.Npad + j], P[((size_t)s1 * 3 + c) * g.Npad + j]};
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int q = 2 * (2 * a + b);
                    acc[q] += e[a].re * p[b].re + e[a].im * p[b].im;
                    acc[q + 1] += e[a].re * p[b].im - e[a].im * p[b].re;
                    acc[8 + q] += w * (p[a].re * p[b].re + p[a].im * p[b].im);
                    acc[9 + q] += w * (p[a].re * p[b].im - p[a].im * p[b].re);
                }
        }
    }
    block_sum_n<16>(acc, sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < 16; ++q) part[((size_t)pr * gridDim.x + blockIdx.x) * 16 + q] = acc[q];
}

// F = sum_j P_j exp(-i k n . r_j) per direction and rhs, FP64.
// Block (dir, rhs pair, chunk): partial sums of F over one chunk of the sites,
// partials[((chunk * nrhs + rhs) * ndir + dir) * 6 + q].  On the lattice the
// phase separates per axis, so the block evaluates n1 + n2 + n3 sincos for
// its direction and each site takes two complex products of table entries.
// PER = false: every rhs takes the same ndir directions, a block serves a
// pair of rhs (same target, same phases).  PER = true: rhs slot r takes
// directions dset[r] * ndir ... dset[r] * ndir + ndir - 1 of nd, one rhs per
// block.
template <bool PER>
__global__ void __launch_bounds__(256) k_ampl(Geo g, double ox, double oy, double oz, double k,
                                              const Cx<double>* __restrict__ P, const double* __restrict__ nd,
                                              double* __restrict__ partials, int ndir, int nrhs,
                                              const int* __restrict__ dset) {
    __shared__ double sh[12 * 4];
    // the phase factors per axis, exp(-i k n_a (a - o_a)) for a = x, y, z at
    // every lattice coordinate of the box: [n1 | n2 | n3]
    extern __shared__ unsigned char smem_raw[];
    Cx<double>* T = reinterpret_cast<Cx<double>*>(smem_raw);
    const int dir = blockIdx.x, r0 = (PER ? 1 : 2) * blockIdx.y, chunk = blockIdx.z;
    const int nr = PER ? 1 : min(2, nrhs - r0);
    const int per = (g.N + gridDim.z - 1) / gridDim.z;
    const int j0 = chunk * per, j1 = min(g.N, j0 + per);
    const size_t di = PER ? (size_t)dset[r0] * ndir + dir : (size_t)dir;
    const double nx = nd[3 * di], ny = nd[3 * di + 1], nz = nd[3 * di + 2];
    const int n12 = g.n1 + g.n2, nt = n12 + g.n3;
    for (int i = threadIdx.x; i < nt; i += blockDim.x) {
        const double a = i < g.n1 ? nx * ((double)i - ox)
                                  : (i < n12 ? ny * ((double)(i - g.n1) - oy) : nz * ((double)(i - n12) - oz));
        double sn, cs;
        sincos(-k * a, &sn, &cs);
        T[i] = Cx<double>{cs, sn};
    }
    __syncthreads();
    double acc[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[i] = 0;
    for (int j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
        const uint32_t s = g.site_xyz[j];
        // exp(-i k n . (r - o)) as the product of the three axis factors
        const Cx<double> ph = (T[s & 1023] * T[g.n1 + ((s >> 10) & 1023)]) * T[n12 + (s >> 20)];
        const double cs = ph.re, sn = ph.im;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= nr) break;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const Cx<double> p = P[((size_t)(r0 + h) * 3 + c) * g.Npad + j];
                acc[6 * h + 2 * c] += p.re * cs - p.im * sn;
                acc[6 * h + 2 * c + 1] += p.re * sn + p.im * cs;
            }
        }
    }
    block_sum_n<12>(acc, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= nr) break;
#pragma unroll
            for (int q = 0; q < 6; ++q)
                partials[(((size_t)chunk * nrhs + r0 + h) * ndir + dir) * 6 + q] = acc[6 * h + q];
        }
}

// Total E and B at points (FP64): the incident wave plus the retarded field
// of every dipole (guide, "Postprocessing: Calculating E and B In or Near the
// Target"); for a dipole p at R = R n from the point, Gaussian units,
//   E = exp(ikR) [k^2/R (p - n (n.p)) + (1/R^3 - ik/R^2) (3 n (n.p) - p)],
//   B = exp(ikR) (k^2/R + ik/R^2) (n x p),
// and the plane wave's B = khat x E_inc.  A point on a site takes no
// contribution from that site.  Block (point, rhs pair) sums the sites; the
// rhs of one target share k, so each site's exp(ikR) serves both.
// out[(rhs * npts + pt) * 12]: E then B, (re, im) per component.
__global__ void __launch_bounds__(256) k_near_field(Geo g, double ox, double oy, double oz,
                                                    const Cx<double>* __restrict__ P,
                                                    const WaveDev* __restrict__ w, const double* __restrict__ pts,
                                                    int npts, int nrhs, double* __restrict__ out) {
    __shared__ double sh[24 * 4];
    const int pt = blockIdx.x, r0 = 2 * blockIdx.y;
    const int nr = min(2, nrhs - r0);
    const double k = w[r0].k;
    const double qx = pts[3 * pt], qy = pts[3 * pt + 1], qz = pts[3 * pt + 2];
    double acc[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) acc[i] = 0;
    for (int j = threadIdx.x; j < g.N; j += blockDim.x) {
        const uint32_t s = g.site_xyz[j];
        const double Rx = qx - ((double)(s & 1023) - ox), Ry = qy - ((double)((s >> 10) & 1023) - oy);
        const double Rz = qz - ((double)(s >> 20) - oz);
        const double R2 = Rx * Rx + Ry * Ry + Rz * Rz;
        if (!(R2 > 1e-18)) continue;  // the point is this site
        const double R = sqrt(R2), iR = 1.0 / R;
        const double n[3] = {Rx * iR, Ry * iR, Rz * iR};
        double sn, cs;
        sincos(k * R, &sn, &cs);
        const Cx<double> ph = {cs, sn};
        const double a = k * k * iR;
        const Cx<double> b = {iR * iR * iR, -k * iR * iR};       // 1/R^3 - ik/R^2
        const Cx<double> cb = ph * Cx<double>{a, k * iR * iR};  // exp(ikR) (k^2/R + ik/R^2)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= nr) break;
            const Cx<double>* Pr = P + (size_t)(r0 + h) * 3 * g.Npad;
            const Cx<double> p[3] = {Pr[j], Pr[g.Npad + j], Pr[2 * g.Npad + j]};
            const Cx<double> np = n[0] * p[0] + n[1] * p[1] + n[2] * p[2];
            const Cx<double> nxp[3] = {n[1] * p[2] - n[2] * p[1], n[2] * p[0] - n[0] * p[2],
                                       n[0] * p[1] - n[1] * p[0]};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const Cx<double> e = ph * (a * (p[c] - n[c] * np) + b * ((3.0 * n[c]) * np - p[c]));
                const Cx<double> bb = cb * nxp[c];
                acc[12 * h + 2 * c] += e.re;
                acc[12 * h + 2 * c + 1] += e.im;
                acc[12 * h + 6 + 2 * c] += bb.re;
                acc[12 * h + 6 + 2 * c + 1] += bb.im;
            }
        }
    }
    block_sum_n<24>(acc, sh);
    if (threadIdx.x != 0) return;
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // unrolled: acc is indexed by constants only
        if (h >= nr) break;
        const WaveDev wv = w[r0 + h];
        double sn, cs;
        sincos(k * (wv.khat[0] * qx + wv.khat[1] * qy + wv.khat[2] * qz), &sn, &cs);
        const Cx<double> ph = {cs, sn};
        Cx<double> ei[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) ei[c] = Cx<double>{wv.e[2 * c], wv.e[2 * c + 1]} * ph;
        const double* kh = wv.khat;
        const Cx<double> bi[3] = {kh[1] * ei[2] - kh[2] * ei[1], kh[2] * ei[0] - kh[0] * ei[2],
                                  kh[0] * ei[1] - kh[1] * ei[0]};
        double* o = out + ((size_t)(r0 + h) * npts + pt) * 12;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o[2 * c] = acc[12 * h + 2 * c] + ei[c].re;
            o[2 * c + 1] = acc[12 * h + 2 * c + 1] + ei[c].im;
            o[6 + 2 * c] = acc[12 * h + 6 + 2 * c] + bi[c].re;
            o[6 + 2 * c + 1] = acc[12 * h + 6 + 2 * c + 1] + bi[c].im;
        }
    }
}

__global__ void k_ampl_reduce(const double* __restrict__ partials, int nchunk, int n, double* __restrict__ F) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double s = 0;
    for (int c = 0; c < nchunk; ++c) s += partials[(size_t)c * n + e];
    F[e] = s;
}

// Previous local field carried to the new incidence direction:
//   esh_j = (1/alpha_prev) P_prev,j exp(i k (khat - khat_prev) . r_j),
// written (each output optional) as the field esh (FP32), as the guess
// P0_j = esh_j / (1/alpha_new) in FP64 (p0) or in FP32 (v32).  p0 may alias
// Pprev: every element is read and written by the same thread.
__device__ __forceinline__ void prev_shift_body(const Geo& g, double ox, double oy, double oz, int rhs,
                                                const Cx<double>* Pprev, const Cx<double>* __restrict__ ainv_prev,
                                                const Cx<double>* __restrict__ ainv_new, const WaveDev& a,
                                                const WaveDev& b, Cx<float>* __restrict__ esh, Cx<double>* p0,
                                                Cx<float>* __restrict__ v32) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < g.Npad; j += gridDim.x * blockDim.x) {
        Cx<double> ph = {0, 0};
        Cx<double> ap = {0, 0}, an = {1, 0};
        if (j < g.N) {
            const uint32_t s = g.site_xyz[j];
            const double x = (double)(s & 1023) - ox, y = (double)((s >> 10) & 1023) - oy, z = (double)(s >> 20) - oz;
            double sn, cs;
            sincos(b.k * ((b.khat[0] - a.khat[0]) * x + (b.khat[1] - a.khat[1]) * y + (b.khat[2] - a.khat[2]) * z),
                   &sn, &cs);
            ph = Cx<double>{cs, sn};
            ap = ainv_prev[(size_t)rhs * g.ncomp + g.site_comp[j]];
            an = ainv_new[(size_t)rhs * g.ncomp + g.site_comp[j]];
        }
        const double dn = an.re * an.re + an.im * an.im;
        for (int c = 0; c < 3; ++c) {
            const size_t i = ((size_t)rhs * 3 + c) * g.Npad + j;
            const Cx<double> e = (ap * Pprev[i]) * ph;
            const Cx<double> q = {(e.re * an.re + e.im * an.im) / dn, (e.im * an.re - e.re * an.im) / dn};
            if (esh) esh[i] = Cx<float>{(float)e.re, (float)e.im};
            if (p0) p0[i] = q;
            if (v32) v32[i] = Cx<float>{(float)q.re, (float)q.im};
        }
    }
}

__global__ void k_prev_shift(Geo g, double ox, double oy, double oz, const Cx<double>* Pprev,
                             const Cx<double>* __restrict__ ainv_prev, const Cx<double>* __restrict__ ainv_new,
                             const WaveDev* __restrict__ wprev, const WaveDev* __restrict__ wnew,
                             Cx<float>* __restrict__ esh, Cx<double>* p0, Cx<float>* __restrict__ v32) {
    const int rhs = blockIdx.y;
    prev_shift_body(g, ox, oy, oz, rhs, Pprev, ainv_prev, ainv_new, wprev[rhs], wnew[rhs], esh, p0, v32);
}

// The history entries of the least-squares guess in one launch: entry e =
// blockIdx.z carried to the new direction into v32 + e ve (FP32).
__global__ void k_prev_shift_hist(Geo g, double ox, double oy, double oz, HistSrc src,
                                  const Cx<double>* __restrict__ ainv_new, const WaveDev* __restrict__ wnew,
                                  Cx<float>* __restrict__ v32, size_t ve) {
    const int rhs = blockIdx.y, e = blockIdx.z;
    prev_shift_body(g, ox, oy, oz, rhs, src.P[e], src.ainv[e], ainv_new, src.w[e][rhs], wnew[rhs], nullptr, nullptr,
                    v32 + e * ve);
}

// Normal equations of min || b - sum_e c_e W_e || per rhs over h <= 4 basis
// vectors: partial sums of <W_e, W_f> (e <= f) and <W_e, b> per block,
// written to partials[rhs][blockIdx.x][14] complex.  W is [h][nrhs][V].
constexpr int MAXH = HIST_MAX;
constexpr int NGRAM = HIST_NGRAM;
__global__ void __launch_bounds__(VT) k_gram_part(int V, int nrhs, int h, const Cx<float>* __restrict__ W,
                                                  const Cx<double>* __restrict__ b, double* __restrict__ partials) {
    const int rhs = blockIdx.y;
    double2 acc[NGRAM];
#pragma unroll
    for (int q = 0; q < NGRAM; ++q) acc[q] = double2{0, 0};
    const size_t es = (size_t)nrhs * V, o = (size_t)rhs * V;
    for (int i = blockIdx.x * VT + threadIdx.x; i < V; i += gridDim.x * VT) {
        Cx<float> w[MAXH];
#pragma unroll
        for (int e = 0; e < MAXH; ++e) w[e] = e < h ? W[e * es + o + i] : Cx<float>{0, 0};
        const Cx<double> bi = b[o + i];
        int q = 0;
#pragma unroll
        for (int e = 0; e < MAXH; ++e) {
#pragma unroll
            for (int f = e; f < MAXH; ++f) acc_dot(acc[q++], w[e], w[f]);
            acc_dot(acc[MAXH * (MAXH + 1) / 2 + e], Cx<double>{w[e].re, w[e].im}, bi);
        }
    }
    // all 2 NGRAM sums with one barrier
    __shared__ double sh[2 * NGRAM * (VT / 64)];
    double v[2 * NGRAM];
#pragma unroll
    for (int q = 0; q < NGRAM; ++q) {
        v[2 * q] = acc[q].x;
        v[2 * q + 1] = acc[q].y;
    }
    block_sum_n<2 * NGRAM>(v, sh);
    if (threadIdx.x == 0) {
        double* out = partials + ((size_t)rhs * gridDim.x + blockIdx.x) * NGRAM * 2;
#pragma unroll
        for (int q = 0; q < 2 * NGRAM; ++q) out[q] = v[q];
    }
}

// x64 = sum_e c[rhs][e] V[e] (FP32 basis, FP64 result); when esh is given also
// the local field esh = (1/alpha) x (FP32); when rf is given also the
// residual field rf = b - sum_e c[rhs][e] W[e] (FP32, W[e] = A V[e]).
__global__ void __launch_bounds__(VT) k_hist_combine(Geo g, int nrhs, int h, const Cx<float>* __restrict__ Vb,
                                                     const Cx<double>* __restrict__ coef, Cx<double>* __restrict__ x64,
                                                     const Cx<double>* __restrict__ ainv, Cx<float>* __restrict__ esh,
                                                     const Cx<float>* __restrict__ Wb, const Cx<double>* __restrict__ b,
                                                     Cx<float>* __restrict__ rf) {
    const int rhs = blockIdx.y;
    const size_t V = (size_t)3 * g.Npad, es = (size_t)nrhs * V, o = (size_t)rhs * V;
    Cx<double> c[MAXH];
#pragma unroll
    for (int e = 0; e < MAXH; ++e) c[e] = e < h ? coef[rhs * MAXH + e] : Cx<double>{0, 0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += (size_t)gridDim.x * blockDim.x) {
        Cx<double> acc = {0, 0};
#pragma unroll
        for (int e = 0; e < MAXH; ++e)
            if (e < h) {
                const Cx<float> v = Vb[e * es + o + i];
                acc = acc + c[e] * Cx<double>{v.re, v.im};
            }
        x64[o + i] = acc;
        if (rf) {
            Cx<double> ax = {0, 0};
#pragma unroll
            for (int e = 0; e < MAXH; ++e)
                if (e < h) {
                    const Cx<float> w = Wb[e * es + o + i];
                    ax = ax + c[e] * Cx<double>{w.re, w.im};
                }
            const Cx<double> rr = b[o + i] - ax;
            rf[o + i] = Cx<float>{(float)rr.re, (float)rr.im};
        }
        if (esh) {
            const int j = (int)(i % g.Npad);
            const Cx<double> a = j < g.N ? ainv[(size_t)rhs * g.ncomp + g.site_comp[j]] : Cx<double>{0, 0};
            const Cx<double> e = a * acc;
            esh[o + i] = Cx<float>{(float)e.re, (float)e.im};
        }
    }
}

}  // namespace

hipError_t launch_prev_shift(const Geo& g, const double* origin, int nrhs, const Cx<double>* Pprev,
                             const Cx<double>* ainv_prev, const Cx<double>* ainv_new, const WaveDev* wprev,
                             const WaveDev* wnew, Cx<float>* esh, Cx<double>* p0, Cx<float>* v32, hipStream_t st) {
    hipLaunchKernelGGL(k_prev_shift, dim3((g.Npad + 255) / 256, nrhs), dim3(256), 0, st, g, origin[0], origin[1],
                       origin[2], Pprev, ainv_prev, ainv_new, wprev, wnew, esh, p0, v32);
    return hipGetLastError();
}

hipError_t launch_prev_shift_hist(const Geo& g, const double* origin, int nrhs, const HistSrc& src,
                                  const Cx<double>* ainv_new, const WaveDev* wnew, Cx<float>* v32, size_t ve,
                                  hipStream_t st) {
    if (src.h < 1 || src.h > HIST_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_prev_shift_hist, dim3((g.Npad + 255) / 256, nrhs, src.h), dim3(256), 0, st, g, origin[0],
                       origin[1], origin[2], src, ainv_new, wnew, v32, ve);
    return hipGetLastError();
}

// blocks of the Gram partial sums per rhs: enough to stream the vectors,
// few enough that the coefficient kernel's reduction over them is short
int gram_blocks(int Npad) { return std::min(256, (3 * Npad + VT - 1) / VT); }

// Least-squares coefficients of the history guess on the device: sum the
// Gram partials of one rhs over the blocks (one wave, fixed order), then solve
// the h x h Hermitian normal equations G c = <W_e, b> in FP64 by a Cholesky
// factorisation G = L L^H, the diagonal raised by 1e-12 of its largest entry
// (positive definite).  Every loop runs to HIST_MAX with the indices known at
// compile time, so the matrices stay in registers.  coef: [rhs][HIST_MAX]
// complex.
__global__ void __launch_bounds__(64) k_proj_coef(int nblk, int h, const double* __restrict__ partials,
                                                  Cx<double>* __restrict__ coef) {
    const int rhs = blockIdx.x;
    double acc[2 * NGRAM];
#pragma unroll
    for (int q = 0; q < 2 * NGRAM; ++q) acc[q] = 0;
    for (int b = threadIdx.x; b < nblk; b += 64) {
        const double* p = partials + ((size_t)rhs * nblk + b) * NGRAM * 2;
#pragma unroll
        for (int q = 0; q < 2 * NGRAM; ++q) acc[q] += p[q];
    }
#pragma unroll
    for (int q = 0; q < 2 * NGRAM; ++q) acc[q] = wave_total(acc[q]);
    if (threadIdx.x != 0) return;
    // G[e][f] = <W_e, W_f> for e <= f (row-major upper triangle), rhs <W_e, b>
    double2 G[MAXH][MAXH], r[MAXH];
    double dmax = 0;
    {
        int q = 0;
#pragma unroll
        for (int e = 0; e < MAXH; ++e)
#pragma unroll
            for (int f = e; f < MAXH; ++f) {
                G[e][f] = make_double2(acc[2 * q], acc[2 * q + 1]);
                ++q;
                if (e == f && e < h) dmax = fmax(dmax, fabs(G[e][e].x));
            }
#pragma unroll
        for (int e = 0; e < MAXH; ++e) r[e] = make_double2(acc[2 * (q + e)], acc[2 * (q + e) + 1]);
    }
    // L (lower, real diagonal): L[i][j] for j <= i
    double2 L[MAXH][MAXH];
    double dg[MAXH];
#pragma unroll
    for (int j = 0; j < MAXH; ++j) {
        if (j >= h) break;
        double d = G[j][j].x + 1e-12 * dmax + 1e-300;
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[j][k].x * L[j][k].x + L[j][k].y * L[j][k].y;
        dg[j] = sqrt(fmax(d, 1e-300));
        const double inv = 1.0 / dg[j];
#pragma unroll
        for (int i = j + 1; i < MAXH; ++i) {
            if (i >= h) break;
            // G[i][j] = conj(G[j][i]); subtract sum_k L[i][k] conj(L[j][k])
            double2 v = make_double2(G[j][i].x, -G[j][i].y);
#pragma unroll
            for (int k = 0; k < j; ++k) {
                const double2 a = L[i][k], c = L[j][k];
                v.x -= a.x * c.x + a.y * c.y;
                v.y -= a.y * c.x - a.x * c.y;
            }
            L[i][j] = make_double2(v.x * inv, v.y * inv);
        }
    }
    // L y = r, then L^H c = y
    double2 y[MAXH], out[MAXH];
#pragma unroll
    for (int i = 0; i < MAXH; ++i) {
        if (i >= h) break;
        double2 v = r[i];
#pragma unroll
        for (int k = 0; k < i; ++k) {
            const double2 a = cmul2(L[i][k], y[k]);
            v = make_double2(v.x - a.x, v.y - a.y);
        }
        y[i] = make_double2(v.x / dg[i], v.y / dg[i]);
    }
#pragma unroll
    for (int i = MAXH - 1; i >= 0; --i) {
        if (i >= h) continue;
        double2 v = y[i];
#pragma unroll
        for (int k = i + 1; k < MAXH; ++k) {
            if (k >= h) break;
            // conj(L[k][i]) * out[k]
            const double2 a = L[k][i], o = out[k];
            v.x -= a.x * o.x + a.y * o.y;
            v.y -= a.x * o.y - a.y * o.x;
        }
        out[i] = make_double2(v.x / dg[i], v.y / dg[i]);
    }
#pragma unroll
    for (int e = 0; e < MAXH; ++e)
        coef[(size_t)rhs * MAXH + e] = e < h ? Cx<double>{out[e].x, out[e].y} : Cx<double>{0, 0};
}

hipError_t launch_proj_coef(int Npad, int nrhs, int h, const double* partials, Cx<double>* coef, hipStream_t st) {
    if (h < 1 || h > MAXH) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_proj_coef, dim3(nrhs), dim3(64), 0, st, gram_blocks(Npad), h, partials, coef);
    return hipGetLastError();
}



hipError_t launch_gram(int Npad, int nrhs, int h, const Cx<float>* W, const Cx<double>* b, double* partials,
                       hipStream_t st) {
    if (h < 1 || h > MAXH) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gram_part, dim3(gram_blocks(Npad), nrhs), dim3(VT), 0, st, 3 * Npad, nrhs, h, W, b,
                       partials);
    return hipGetLastError();
}

hipError_t launch_hist_combine(const Geo& g, int nrhs, int h, const Cx<float>* V, const Cx<double>* coef,
                               Cx<double>* x64, const Cx<double>* ainv, Cx<float>* esh, const Cx<float>* W,
                               const Cx<double>* b, Cx<float>* rf, hipStream_t st) {
    if (h < 1 || h > MAXH) return hipErrorInvalidValue;
    if (rf && (!W || !b)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_hist_combine, dim3((3 * g.Npad + VT - 1) / VT, nrhs), dim3(VT), 0, st, g, nrhs, h, V, coef,
                       x64, ainv, esh, W, b, rf);
    return hipGetLastError();
}

int vec_blocks(int Npad) { return (3 * Npad + VB - 1) / VB; }

template <class T>
hipError_t launch_einc(const Geo& g, const double* o, const WaveDev* w, int nrhs, Cx<T>* E, hipStream_t st) {
    hipLaunchKernelGGL((k_einc<T>), dim3((g.Npad + VT - 1) / VT, nrhs), dim3(VT), 0, st, g, o[0], o[1], o[2], w, E);
    return hipGetLastError();
}
template <class T>
hipError_t launch_fill(Cx<T>* p, size_t n, hipStream_t st) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL((k_fillv<T>), dim3(1024), dim3(256), 0, st, p, n);
    return hipGetLastError();
}
hipError_t launch_fill_int(int* p, int v, size_t n, hipStream_t st) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_filli, dim3(64), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

template <class T>
hipError_t launch_bicg_p(int Npad, int nrhs, Cx<T>* p, const Cx<T>* r, const Cx<T>* v, Cx<T>* rhat,
                         const BiState* s, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_bicg_p<T>), dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, st, 3 * Npad, p, r, v, rhat, s,
                       active);
    return hipGetLastError();
}
template <class T>
hipError_t launch_dot(int Npad, int nrhs, int npair, const Cx<T>* a0, const Cx<T>* b0, const Cx<T>* a1,
                      const Cx<T>* b1, double* partials, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_dot<T>), dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, st, 3 * Npad, npair, a0, b0, a1, b1,
                       partials, active);
    return hipGetLastError();
}
template <class T>
hipError_t launch_bicg_s(int Npad, int nrhs, Cx<T>* s, const Cx<T>* r, const Cx<T>* v, const BiState* st_,
                         const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_bicg_s<T>), dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, st, 3 * Npad, s, r, v, st_, active);
    return hipGetLastError();
}
template <class T>
hipError_t launch_bicg_xr(int Npad, int nrhs, Cx<T>* x, Cx<T>* r, const Cx<T>* p, const Cx<T>* s, const Cx<T>* t,
                          const Cx<T>* rhat, const BiState* st_, double* partials, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_bicg_xr<T>), dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, st, 3 * Npad, x, r, p, s, t, rhat,
                       st_, partials, active);
    return hipGetLastError();
}
hipError_t launch_scalars(int which, int nblk, int nrhs, BiState* s, const double* partials, int* active, int kpar,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_scalars, dim3(nrhs), dim3(SCALAR_THREADS), 0, st, which, nblk, s, partials, active, kpar);
    return hipGetLastError();
}
template <class T>
hipError_t launch_bicg_upd(int Npad, int nrhs, Cx<T>* x, Cx<T>* r, const Cx<T>* p, Cx<T>* pout, const Cx<T>* v,
                           Cx<T>* rhat, const Cx<T>* s, const Cx<T>* t, const BiState* st, const int* active,
                           hipStream_t stream) {
    hipLaunchKernelGGL((k_bicg_upd<T>), dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, stream, 3 * Npad, x, r, p, pout, v,
                       rhat, s, t, st, active);
    return hipGetLastError();
}
template hipError_t launch_bicg_upd<float>(int, int, Cx<float>*, Cx<float>*, const Cx<float>*, Cx<float>*,
                                           const Cx<float>*, Cx<float>*, const Cx<float>*, const Cx<float>*,
                                           const BiState*, const int*, hipStream_t);
template hipError_t launch_bicg_upd<double>(int, int, Cx<double>*, Cx<double>*, const Cx<double>*, Cx<double>*,
                                            const Cx<double>*, Cx<double>*, const Cx<double>*, const Cx<double>*,
                                            const BiState*, const int*, hipStream_t);
template <class T>
hipError_t launch_bicg_flush(int Npad, int nrhs, Cx<T>* x, Cx<T>* r, const Cx<T>* p0, const Cx<T>* p1,
                             const Cx<T>* s, const Cx<T>* t, BiState* st, hipStream_t stream) {
    hipLaunchKernelGGL((k_bicg_flush<T>), dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, stream, 3 * Npad, x, r, p0, p1,
                       s, t, st);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_clear_pend, dim3((nrhs + 255) / 256), dim3(256), 0, stream, st, nrhs);
    return hipGetLastError();
}
template hipError_t launch_bicg_flush<float>(int, int, Cx<float>*, Cx<float>*, const Cx<float>*, const Cx<float>*,
                                             const Cx<float>*, const Cx<float>*, BiState*, hipStream_t);
template hipError_t launch_bicg_flush<double>(int, int, Cx<double>*, Cx<double>*, const Cx<double>*,
                                              const Cx<double>*, const Cx<double>*, const Cx<double>*, BiState*,
                                              hipStream_t);
template <class T>
hipError_t launch_bicg_init(int Npad, int nrhs, const Cx<T>* b, Cx<T>* x, Cx<T>* r, Cx<T>* rhat, Cx<T>* p, Cx<T>* v,
                            hipStream_t st) {
    hipLaunchKernelGGL((k_bicg_init<T>), dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, st, 3 * Npad, b, x, r, rhat, p, v);
    return hipGetLastError();
}
hipError_t launch_state_init(int Npad, int nrhs, BiState* s, const double* partials, const double* tol_rel2,
                             const int* maxit, int* active, int frs, double* trace, int tcap, hipStream_t st) {
    hipLaunchKernelGGL(k_state_init, dim3(nrhs), dim3(256), 0, st, vec_blocks(Npad), s, partials, tol_rel2, maxit,
                       active, frs, trace, tcap);
    return hipGetLastError();
}
hipError_t launch_l2_state_init(int Npad, int nrhs, BiState* s, const double* partials, const double* tol_rel2,
                                const int* maxit, int* active, int frs, double* trace, int tcap, hipStream_t st) {
    hipLaunchKernelGGL(k_l2_state_init, dim3(nrhs), dim3(256), 0, st, vec_blocks(Npad), s, partials, tol_rel2, maxit,
                       active, frs, trace, tcap);
    return hipGetLastError();
}
hipError_t launch_l2_scalars(int which, int nblk, int nrhs, BiState* s, const double* partials, int* active,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_l2_scalars, dim3(nrhs), dim3(SCALAR_THREADS), 0, st, which, nblk, s, partials, active);
    return hipGetLastError();
}
template <class T>
hipError_t launch_l2_update(int step, int Npad, int nrhs, Cx<T>* x, Cx<T>* r0, Cx<T>* rt, Cx<T>* u0, Cx<T>* u1,
                            const Cx<T>* u2, Cx<T>* r1, const Cx<T>* r2, const BiState* s, double* partials,
                            const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_l2_update<T>), dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, st, step, 3 * Npad, x, r0, rt, u0,
                       u1, u2, r1, r2, s, partials, active);
    return hipGetLastError();
}
template <class T>
hipError_t launch_l2_mrdot(int Npad, int nrhs, const Cx<T>* r0, const Cx<T>* r1, const Cx<T>* r2, double* partials,
                           const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_l2_mrdot<T>), dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, st, 3 * Npad, r0, r1, r2, partials,
                       active);
    return hipGetLastError();
}
template hipError_t launch_l2_update<float>(int, int, int, Cx<float>*, Cx<float>*, Cx<float>*, Cx<float>*, Cx<float>*,
                                            const Cx<float>*, Cx<float>*, const Cx<float>*, const BiState*, double*,
                                            const int*, hipStream_t);
template hipError_t launch_l2_update<double>(int, int, int, Cx<double>*, Cx<double>*, Cx<double>*, Cx<double>*,
                                             Cx<double>*, const Cx<double>*, Cx<double>*, const Cx<double>*,
                                             const BiState*, double*, const int*, hipStream_t);
template hipError_t launch_l2_mrdot<float>(int, int, const Cx<float>*, const Cx<float>*, const Cx<float>*, double*,
                                           const int*, hipStream_t);
template hipError_t launch_l2_mrdot<double>(int, int, const Cx<double>*, const Cx<double>*, const Cx<double>*,
                                            double*, const int*, hipStream_t);
template <class T>
hipError_t launch_aniso_diag(const Geo& g, int nrhs, const Cx<T>* x, Cx<T>* y, const Cx<T>* tens, int sgn,
                             hipStream_t st) {
    hipLaunchKernelGGL((k_aniso_diag<T>), dim3((g.N + 255) / 256, nrhs), dim3(256), 0, st, g, x, y, tens, (T)sgn);
    return hipGetLastError();
}
template hipError_t launch_aniso_diag<float>(const Geo&, int, const Cx<float>*, Cx<float>*, const Cx<float>*, int,
                                             hipStream_t);
template hipError_t launch_aniso_diag<double>(const Geo&, int, const Cx<double>*, Cx<double>*, const Cx<double>*, int,
                                              hipStream_t);
hipError_t launch_aniso_abs(const Geo& g, int nrhs, const Cx<double>* P, const Cx<double>* tens, double* partials,
                            double* out, hipStream_t st) {
    const int nblk = vec_blocks(g.Npad);
    hipLaunchKernelGGL(k_aniso_abs, dim3(nblk, nrhs), dim3(VT), 0, st, g, P, tens, partials);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_norm2_final, dim3(nrhs), dim3(256), 0, st, nblk, partials, out);
    return hipGetLastError();
}
hipError_t launch_demote(int Npad, int nrhs, const Cx<double>* r64, Cx<float>* r32, const double* scale,
                         const int* mask, hipStream_t st) {
    hipLaunchKernelGGL(k_demote, dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, st, 3 * Npad, r64, r32, scale, mask);
    return hipGetLastError();
}
__global__ void k_demote_table(int n, const Cx<double>* __restrict__ in, Cx<float>* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = Cx<float>{(float)in[i].re, (float)in[i].im};
}
hipError_t launch_demote_table(int n, const Cx<double>* in, Cx<float>* out, hipStream_t st) {
    hipLaunchKernelGGL(k_demote_table, dim3((n + 255) / 256), dim3(256), 0, st, n, in, out);
    return hipGetLastError();
}
hipError_t launch_promote_add(int Npad, int nrhs, Cx<double>* x64, const Cx<float>* d32, const double* scale,
                              const int* mask, const BiState* bst, hipStream_t st) {
    hipLaunchKernelGGL(k_promote_add, dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, st, 3 * Npad, x64, d32, scale, mask,
                       bst);
    return hipGetLastError();
}
template <class T>
hipError_t launch_axpy_masked(int Npad, int nrhs, Cx<T>* x, const Cx<T>* d, const int* mask, const BiState* bst,
                              hipStream_t st) {
    hipLaunchKernelGGL((k_axpy_masked<T>), dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, st, 3 * Npad, x, d, mask, bst);
    return hipGetLastError();
}
template <class T>
hipError_t launch_norm2(int Npad, int nrhs, const Cx<T>* v, double* partials, double* out, hipStream_t st) {
    hipLaunchKernelGGL((k_norm2_part<T>), dim3(vec_blocks(Npad), nrhs), dim3(VT), 0, st, 3 * Npad, v, partials);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_norm2_final, dim3(nrhs), dim3(256), 0, st, vec_blocks(Npad), partials, out);
    return hipGetLastError();
}
template <class T>
hipError_t launch_from_abi(const Geo& g, int nrhs, const Cx<double>* in, Cx<T>* out, hipStream_t st) {
    hipLaunchKernelGGL((k_from_abi<T>), dim3((g.Npad + 255) / 256, nrhs), dim3(256), 0, st, g.N, g.Npad, g.perm, in,
                       out);
    return hipGetLastError();
}
template <class T>
hipError_t launch_to_abi(const Geo& g, int nrhs, const Cx<T>* in, Cx<double>* out, hipStream_t st) {
    hipLaunchKernelGGL((k_to_abi<T>), dim3((g.N + 255) / 256, nrhs), dim3(256), 0, st, g.N, g.Npad, g.perm, in, out);
    return hipGetLastError();
}
hipError_t launch_xsec(const Geo& g, int nrhs, const Cx<double>* E, const Cx<double>* P, const Cx<double>* ainv,
                       double k3, double* partials, double* out, hipStream_t st) {
    const int nblk = vec_blocks(g.Npad);
    hipLaunchKernelGGL(k_xsec_part, dim3(nblk, nrhs), dim3(VT), 0, st, g, E, P, ainv, k3, partials);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_xsec_final, dim3(nrhs), dim3(256), 0, st, nblk, partials, out);
    return hipGetLastError();
}
int xsec_pair_blocks(int N) { return std::max(1, std::min(256, (N + 255) / 256)); }
hipError_t launch_xsec_pair(const Geo& g, int npairs, const Cx<double>* E, const Cx<double>* P,
                            const Cx<double>* ainv, double k3, const int* slots, double* part, hipStream_t st) {
    hipLaunchKernelGGL(k_xsec_pair, dim3(xsec_pair_blocks(g.N), npairs), dim3(256), 0, st, g, E, P, ainv, k3, slots,
                       part);
    return hipGetLastError();
}
int ampl_chunks(int ndir, int nrhs, int N) {
    const int want = (2048 + ndir * nrhs - 1) / (ndir * nrhs);
    return std::max(1, std::min({64, want, (N + 1023) / 1024}));
}
hipError_t launch_near_field(const Geo& g, const double* o, int nrhs, const Cx<double>* P, const WaveDev* w,
                             const double* pts, int npts, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_near_field, dim3(npts, (nrhs + 1) / 2), dim3(256), 0, st, g, o[0], o[1], o[2], P, w, pts,
                       npts, nrhs, out);
    return hipGetLastError();
}
hipError_t launch_ampl(const Geo& g, const double* o, double k, int nrhs, const Cx<double>* P, int ndir,
                       const double* ndirs, Cx<double>* F, double* partials, hipStream_t st, const int* dset) {
    const int nc = ampl_chunks(ndir, nrhs, g.N);
    const size_t lds = (size_t)(g.n1 + g.n2 + g.n3) * sizeof(Cx<double>);  // at most 3 x 1023 entries
    if (dset)
        hipLaunchKernelGGL(k_ampl<true>, dim3(ndir, nrhs, nc), dim3(256), lds, st, g, o[0], o[1], o[2], k, P, ndirs,
                           partials, ndir, nrhs, dset);
    else
        hipLaunchKernelGGL(k_ampl<false>, dim3(ndir, (nrhs + 1) / 2, nc), dim3(256), lds, st, g, o[0], o[1], o[2], k,
                           P, ndirs, partials, ndir, nrhs, dset);
    HIP_TRY(hipGetLastError());
    const int n = nrhs * ndir * 6;
    hipLaunchKernelGGL(k_ampl_reduce, dim3((n + 255) / 256), dim3(256), 0, st, partials, nc, n,
                       reinterpret_cast<double*>(F));
    return hipGetLastError();
}

#define INST(T)                                                                                                      \
    template hipError_t launch_einc<T>(const Geo&, const double*, const WaveDev*, int, Cx<T>*, hipStream_t);         \
    template hipError_t launch_fill<T>(Cx<T>*, size_t, hipStream_t);                                                 \
    template hipError_t launch_bicg_p<T>(int, int, Cx<T>*, const Cx<T>*, const Cx<T>*, Cx<T>*, const BiState*,      \
                                         const int*, hipStream_t);                                                   \
    template hipError_t launch_dot<T>(int, int, int, const Cx<T>*, const Cx<T>*, const Cx<T>*, const Cx<T>*, double*, \
                                      const int*, hipStream_t);                                                      \
    template hipError_t launch_bicg_s<T>(int, int, Cx<T>*, const Cx<T>*, const Cx<T>*, const BiState*, const int*,   \
                                         hipStream_t);                                                               \
    template hipError_t launch_bicg_xr<T>(int, int, Cx<T>*, Cx<T>*, const Cx<T>*, const Cx<T>*, const Cx<T>*,        \
                                          const Cx<T>*, const BiState*, double*, const int*, hipStream_t);           \
    template hipError_t launch_bicg_init<T>(int, int, const Cx<T>*, Cx<T>*, Cx<T>*, Cx<T>*, Cx<T>*, Cx<T>*,          \
                                            hipStream_t);                                                            \
    template hipError_t launch_axpy_masked<T>(int, int, Cx<T>*, const Cx<T>*, const int*, const BiState*,           \
                                              hipStream_t);                                                          \
    template hipError_t launch_norm2<T>(int, int, const Cx<T>*, double*, double*, hipStream_t);                      \
    template hipError_t launch_from_abi<T>(const Geo&, int, const Cx<double>*, Cx<T>*, hipStream_t);                 \
    template hipError_t launch_to_abi<T>(const Geo&, int, const Cx<T>*, Cx<double>*, hipStream_t);
INST(float)
INST(double)
