// Internal interface between the host runtime (api.hip) and the kernel
// translation units of the DDA library.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dda_device.h"

// Geometry of one target on the device.  Sites are ordered by linear box index;
// site_xyz packs (x | y << 10 | z << 20); plane_start[z] is the first site of
// plane z (n3 + 1 entries).
// Sites are stored plane by plane (z), and inside a plane grouped by parity
// class q = 2 (y % 2) + (x % 2), scan order (y, then x) inside a class.
struct Geo {
    int n1, n2, n3;
    int N, Npad;
    int ncomp;
    const int* plane_start;    // [n3 + 1]: first site of plane z
    const int* class_start;    // [4 n3 + 1]: first site of class q of plane z at 4 z + q
    const uint32_t* site_xyz;  // x | y << 10 | z << 20
    const uint8_t* site_comp;  // 0-based composition index
    const int* perm;           // [N]: position of each stored site in the (z, y, x) scan order
    // n = 64: z-pass tile order per XCD for tiles of 16 and 32 columns and
    // for 16-column tiles of the class-grouped slab, [8][tiles / 8]; the
    // tiles that share tensor-spectrum columns through the x and y folds are
    // adjacent on one XCD (nullptr for other boxes)
    const int* ztiles16;
    const int* ztiles32;
    const int* ztiles16g;
    // n = 128: the same for 8-column tiles (two-factor 16 x 8 z pass), in
    // the row layout and in the class-grouped layout
    const int* ztiles8;
    const int* ztiles8g;
};

// Twiddle tables of one target: f_i[k] = exp(-2 pi i k / n_i) (k < n_i) and
// h_i[x] = exp(-2 pi i x / (2 n_i)) (x < n_i), the pre-twiddles of the
// frequency-parity split of the doubled axis.
template <class T>
struct Tw {
    const Cx<T>* f1;
    const Cx<T>* f2;
    const Cx<T>* f3;
    const Cx<T>* h1;
    const Cx<T>* h2;
    const Cx<T>* h3;
};

// Per right-hand-side state of BiCGstab (device memory).
struct BiState {
    double rho[2], alpha[2], omega[2], beta[2];
    double rr;     // ||r||^2 (recursive residual)
    double tol2;   // stop when rr <= tol2
    int it, maxit, restart, conv;
    // fused iteration: the update x += alpha p + omega s, r = s - omega t of
    // the last completed iteration is still to be applied (by the next
    // iteration's first pass, or by the flush after the solve); p is in the
    // direction buffer pbuf (0 or 1)
    int pend, pbuf;
    // test hook: a breakdown restart is forced after every frs-th iteration
    // (0: never); trace: when non-null, rr after iteration i is written to
    // trace[i - 1] for i <= tcap
    int frs, tcap;
    double* trace;
    // BiCGstab(2): <rt, r0> for the next cycle (0, 1), the polynomial
    // coefficients gamma_1 (2, 3) and gamma_2 (4, 5) of the last MR step
    double ex[6];
};

// Launch shapes of the three matvec passes for one target and precision.
struct MvShape {
    int fused;       // 1: xy planes in LDS; 0: line kernels through global memory
    int nth_plane;   // threads of the xy-plane kernels
    int nth_z;       // threads of the z-pass kernel
    int tx;          // columns per z-pass block
    int lines_tl;    // lines per block in the line-kernel fallback
    int nth_lines;
    int ct;          // bit 0: specialised plane kernels, bit 1: specialised z pass (cubic boxes),
                     // bit 2: two-factor inverse plane pass (n = 64, with bit 0), bit 3: class-grouped
                     // slab, the quadrant pre-combination done by the z pass (n = 64, bits 0, 1, zrb 3)
    int zrb;         // specialised z pass variant: 0 = one rhs per block, 1 = loop over up to 8 rhs per
                     // block with the spectrum in registers, 2 = two-factor 8 x 8 pass (n = 64),
                     // 3 = two-factor pass with one frequency parity per block half (n = 64),
                     // 4 = two-factor 16 x 8 pass with one parity per block half (n = 128, FP32)
};

// Optional BiCGstab vector update fused into the first matvec pass
// (specialised plane kernels only): mode 2 = s = r - alpha v (alpha from st)
// into pout, and the transformed vector is s; mode 0 = none.
struct MvUpd {
    int mode;
    const void* r;
    const void* v;
    void* pout;
    BiState* st;
    const double* part;  // mode 2: block partials of <rhat, v> (alpha is formed in the pass)
};

// Optional inner products fused into the last matvec pass (specialised plane
// kernels only): dot = 1 -> <w, y> in slot 0; dot = 2 -> <y, x>, <y, y>;
// dot = 3 -> <y, x> (slot 0), (<y, y>, <x, x>) (slot 1), <w, x> (slot 2),
// <w, y> (slot 3).
struct MvDot {
    int dot;
    const void* w;
    double* partials;
};

enum { MV_AX = 0, MV_RESID = 1 };

// largest slab of one chunk of a batched matvec (fits the last-level cache
// with the chunk's vectors and the spectrum)
constexpr size_t MV_CHUNK_BYTES = (size_t)208 << 20;

// ---- matvec / FFT launchers (kernels_fft.hip) ----
template <class T>
hipError_t launch_matvec(const Geo& g, const Tw<T>& tw, const FftPlan* plans, const MvShape& sh, int nrhs,
                         const Cx<T>* x, Cx<T>* y, const Cx<T>* b, Cx<T>* slab, const Cx<T>* ghat,
                         const Cx<T>* ainv, const int* active, int mode, hipStream_t st, MvDot dot = MvDot{0, nullptr, nullptr},
                         MvUpd upd = MvUpd{0, nullptr, nullptr, nullptr, nullptr, nullptr});
// Individual passes (for per-pass profiling).
template <class T>
hipError_t launch_pass(int which, const Geo& g, const Tw<T>& tw, const FftPlan* plans, const MvShape& sh,
                       int nrhs, const Cx<T>* x, Cx<T>* y, const Cx<T>* b, Cx<T>* slab, const Cx<T>* ghat,
                       const Cx<T>* ainv, const int* active, int mode, hipStream_t st,
                       MvDot dot = MvDot{0, nullptr, nullptr},
                       MvUpd upd = MvUpd{0, nullptr, nullptr, nullptr, nullptr, nullptr});
// Shared-memory bytes and feasibility of a shape.
template <class T>
bool matvec_shape_ok(const Geo& g, const FftPlan* plans, const MvShape& sh);

// Spectrum of the interaction tensor: fills the octant arrays (6 components,
// scaled by 1/(M1 M2 M3)) in FP64 and, when g32 != nullptr, an FP32 copy.
// work must hold 48 * n1 n2 n3 complex doubles.
// The tensor spectrum with the 6 components of each frequency adjacent,
// gz[i * 6 + q] = gh[q * cs + i] (read by the two-factor z pass); hx = n/2 > 0
// also permutes the x columns of each parity half into the group order of the
// class-grouped slab (hx = 0: no permutation).
template <class T>
hipError_t launch_green_interleave(const Cx<T>* gh, Cx<T>* gz, size_t cs, int hx, hipStream_t st);
hipError_t launch_green(const Geo& g, const Tw<double>& tw, const FftPlan* plans, double kd, Cx<double>* work,
                        Cx<double>* g64, Cx<float>* g32, hipStream_t st);

inline size_t ghat_octant_elems(int n1, int n2, int n3) {
    return (size_t)6 * (2 * (n1 / 2 + 1)) * (2 * (n2 / 2 + 1)) * (2 * (n3 / 2 + 1));
}

// ---- vector kernels (kernels_vec.hip) ----
struct WaveDev {
    double khat[3];
    double e[6];
    double k;
    double pad;
};

template <class T>
hipError_t launch_einc(const Geo& g, const double* origin3, const WaveDev* w, int nrhs, Cx<T>* E, hipStream_t st);
template <class T>
hipError_t launch_fill(Cx<T>* p, size_t n, hipStream_t st);
hipError_t launch_fill_int(int* p, int v, size_t n, hipStream_t st);

// BiCGstab pieces; vectors are [nrhs][3][Npad]; partials [nrhs][4][nblk] double2.
int vec_blocks(int Npad);
template <class T>
hipError_t launch_bicg_p(int Npad, int nrhs, Cx<T>* p, const Cx<T>* r, const Cx<T>* v, Cx<T>* rhat,
                         const BiState* s, const int* active, hipStream_t st);
template <class T>
hipError_t launch_dot(int Npad, int nrhs, int npair, const Cx<T>* a0, const Cx<T>* b0, const Cx<T>* a1,
                      const Cx<T>* b1, double* partials, const int* active, hipStream_t st);
template <class T>
hipError_t launch_bicg_s(int Npad, int nrhs, Cx<T>* s, const Cx<T>* r, const Cx<T>* v, const BiState* st_,
                         const int* active, hipStream_t st);
template <class T>
hipError_t launch_bicg_xr(int Npad, int nrhs, Cx<T>* x, Cx<T>* r, const Cx<T>* p, const Cx<T>* s,
                          const Cx<T>* t, const Cx<T>* rhat, const BiState* st_, double* partials,
                          const int* active, hipStream_t st);
// which: 0 alpha, 1 omega, 2 rho/convergence; nblk partials per rhs and slot
hipError_t launch_scalars(int which, int nblk, int nrhs, BiState* s, const double* partials, int* active, int kpar,
                          hipStream_t st);
// Apply the pending update of a fused iteration (BiState.pend): x += alpha p +
// omega s, r = s - omega t with p in p0 or p1 by BiState.pbuf; clears pend.
// Fused iteration's direction update as a separate stream over all sites
// (what the forward pass does in mode 3), p' into pout.
template <class T>
hipError_t launch_bicg_upd(int Npad, int nrhs, Cx<T>* x, Cx<T>* r, const Cx<T>* p, Cx<T>* pout, const Cx<T>* v,
                           Cx<T>* rhat, const Cx<T>* s, const Cx<T>* t, const BiState* st, const int* active,
                           hipStream_t stream);
template <class T>
hipError_t launch_bicg_flush(int Npad, int nrhs, Cx<T>* x, Cx<T>* r, const Cx<T>* p0, const Cx<T>* p1,
                             const Cx<T>* s, const Cx<T>* t, BiState* st, hipStream_t stream);
template <class T>
hipError_t launch_bicg_init(int Npad, int nrhs, const Cx<T>* b, Cx<T>* x, Cx<T>* r, Cx<T>* rhat, Cx<T>* p,
                            Cx<T>* v, hipStream_t st);
// state init from partials holding <r,r> in slot 0: rho = rr, restart = 1
// frs: forced-restart period (0 = none); trace: nrhs x tcap doubles or null
hipError_t launch_state_init(int Npad, int nrhs, BiState* s, const double* partials, const double* tol_rel2,
                             const int* maxit, int* active, int frs, double* trace, int tcap, hipStream_t st);

// BiCGstab(2) (the guide's PBCGS2) on vectors [rhs][3][Npad]: x, r0, rt
// (shadow residual), u0, u1, u2, r1, r2.  BiState fields: rho = rho0, alpha,
// omega, beta as in BiCGstab; restart = the cycle in progress started over
// (rt := r0), pend = a restart is due at the next cycle; ex as above.
// State from <r0, r0> in partials slot 0: rho0 = 1, alpha = 0, omega = 1.
hipError_t launch_l2_state_init(int Npad, int nrhs, BiState* s, const double* partials, const double* tol_rel2,
                                const int* maxit, int* active, int frs, double* trace, int tcap, hipStream_t st);
// which: 0 cycle start (beta of the first BiCG step), 1 alpha = rho0 / <rt, u> (slot 0),
// 2 beta of the second BiCG step from <rt, r1> (slot 0), 3 the MR coefficients
// from slots 0..3 as the inverse pass's DOT = 3 leaves them with x = r1, y = r2,
// w = r0, 4 cycle end from <rt, r0> (slot 0) and ||r0||^2 (slot 1)
hipError_t launch_l2_scalars(int which, int nblk, int nrhs, BiState* s, const double* partials, int* active,
                             hipStream_t st);
// step 1: u0 = r0 - beta u0 (rt = r0 on restart); 2: r0 -= alpha u1, x += alpha u0;
// 3: u0 = r0 - beta u0, u1 = r1 - beta u1; 4: r0 -= alpha u1, r1 -= alpha u2, x += alpha u0;
// 5: x += g1 r0 + g2 r1, r0 -= g1 r1 + g2 r2, u0 -= g1 u1 + g2 u2 with partials
// <rt, r0> (slot 0) and ||r0||^2 (slot 1)
template <class T>
hipError_t launch_l2_update(int step, int Npad, int nrhs, Cx<T>* x, Cx<T>* r0, Cx<T>* rt, Cx<T>* u0, Cx<T>* u1,
                            const Cx<T>* u2, Cx<T>* r1, const Cx<T>* r2, const BiState* s, double* partials,
                            const int* active, hipStream_t st);
// The MR inner products in the inverse pass's DOT = 3 layout: slot 0 <r2, r1>,
// slot 1 (||r2||^2, ||r1||^2), slot 2 <r0, r1>, slot 3 <r0, r2> (<a, b> = a^H b)
template <class T>
hipError_t launch_l2_mrdot(int Npad, int nrhs, const Cx<T>* r0, const Cx<T>* r1, const Cx<T>* r2, double* partials,
                           const int* active, hipStream_t st);

// Anisotropic compositions.  tens: [rhs][ncomp][6] complex (xx, xy, xz, yy,
// yz, zz) of the symmetric tensor 1/alpha, zero for isotropic compositions.
// y += sgn T x at every site (sgn = +1 for A x, -1 for the residual b - A x);
// out[rhs] = sum over sites of Im(P . conj(T) P^*) (the tensor part of the
// absorption sum).
template <class T>
hipError_t launch_aniso_diag(const Geo& g, int nrhs, const Cx<T>* x, Cx<T>* y, const Cx<T>* tens, int sgn,
                             hipStream_t st);
hipError_t launch_aniso_abs(const Geo& g, int nrhs, const Cx<double>* P, const Cx<double>* tens, double* partials,
                            double* out, hipStream_t st);

// Mixed precision helpers.
// r32 = r64 * scale[rhs] (scale = 1/||r||); x64 += (1/scale[rhs]) * d32
hipError_t launch_demote(int Npad, int nrhs, const Cx<double>* r64, Cx<float>* r32, const double* scale,
                         const int* mask, hipStream_t st);
// out[i] = in[i] rounded to FP32, i < n (a 1/alpha table)
hipError_t launch_demote_table(int n, const Cx<double>* in, Cx<float>* out, hipStream_t st);
// Both skip a rhs whose inner solve ended with a non-finite recursive
// residual (st[rhs].rr), so that x64 keeps its last finite value.
hipError_t launch_promote_add(int Npad, int nrhs, Cx<double>* x64, const Cx<float>* d32, const double* scale,
                              const int* mask, const BiState* st, hipStream_t stream);
template <class T>
hipError_t launch_axpy_masked(int Npad, int nrhs, Cx<T>* x, const Cx<T>* d, const int* mask, const BiState* st,
                              hipStream_t stream);
// per-rhs ||v||^2 into out[rhs] (double), two-stage
template <class T>
hipError_t launch_norm2(int Npad, int nrhs, const Cx<T>* v, double* partials, double* out, hipStream_t st);

// Layout conversion between the ABI ([rhs][N][3] complex128, sites in
// (z, y, x) scan order) and the device layout ([rhs][3][Npad], stored order).
template <class T>
hipError_t launch_from_abi(const Geo& g, int nrhs, const Cx<double>* in, Cx<T>* out, hipStream_t st);
template <class T>
hipError_t launch_to_abi(const Geo& g, int nrhs, const Cx<T>* in, Cx<double>* out, hipStream_t st);

// Cross-section sums: out[rhs] = {sum Im(E^* . P), sum |P|^2 * (-Im ainv_c - (2/3) k^3),
// sum Re(E^* . P)}.
hipError_t launch_xsec(const Geo& g, int nrhs, const Cx<double>* E, const Cx<double>* P, const Cx<double>* ainv,
                       double k3, double* partials, double* out, hipStream_t st);
// Pair sums of the cross sections of combined solutions: for each pair of
// slots (slots[2p], slots[2p+1]), xsec_pair_blocks(N) block partials of the
// 16 doubles S_ab = sum conj(E_a) . P_b, G_ab = sum w conj(P_a) . P_b
// (w = -Im ainv - (2/3) k^3) into part[(p * nblk + blk) * 16 + q].
int xsec_pair_blocks(int N);
hipError_t launch_xsec_pair(const Geo& g, int npairs, const Cx<double>* E, const Cx<double>* P,
                            const Cx<double>* ainv, double k3, const int* slots, double* part, hipStream_t st);
// Amplitude sums F[rhs][dir][3] = sum_j P_j exp(-i k n . r_j) (FP64).
// Site chunks per (direction, rhs) of the amplitude sums; partials holds
// ampl_chunks * nrhs * ndir * 6 doubles.
int ampl_chunks(int ndir, int nrhs, int N);
// E and B at npts points (TF, lattice units from the origin o) for nrhs
// solutions P ([nrhs][3][Npad]) and their waves; out [nrhs][npts][12].
hipError_t launch_near_field(const Geo& g, const double* o, int nrhs, const Cx<double>* P, const WaveDev* w,
                             const double* pts, int npts, double* out, hipStream_t st);
hipError_t launch_ampl(const Geo& g, const double* o, double k, int nrhs, const Cx<double>* P, int ndir,
                       const double* ndirs, Cx<double>* F, double* partials, hipStream_t st,
                       const int* dset = nullptr);

hipError_t configure_fft_kernels();

// Previous local field (1/alpha_prev) P_prev carried to the new incidence
// direction: optional outputs esh (the field, FP32), p0 = esh / (1/alpha_new)
// (FP64, may alias Pprev) and v32 (the same guess in FP32).
hipError_t launch_prev_shift(const Geo& g, const double* origin, int nrhs, const Cx<double>* Pprev,
                             const Cx<double>* ainv_prev, const Cx<double>* ainv_new, const WaveDev* wprev,
                             const WaveDev* wnew, Cx<float>* esh, Cx<double>* p0, Cx<float>* v32, hipStream_t st);
// Least-squares combination of up to 4 basis vectors per rhs: block partials
// [rhs][gram_blocks][14] complex of <W_e, W_f> (e <= f, row-major upper
// triangle of the 4 x 4 matrix) then <W_e, b>; W, V are [h][nrhs][3][Npad].
constexpr int HIST_MAX = 4;
constexpr int HIST_NGRAM = HIST_MAX * (HIST_MAX + 1) / 2 + HIST_MAX;
// the h stored solutions of a group, their 1/alpha tables and waves
struct HistSrc {
    const Cx<double>* P[HIST_MAX];
    const Cx<double>* ainv[HIST_MAX];
    const WaveDev* w[HIST_MAX];
    int h;
};
// v32 + e ve = entry e carried to the new direction (as launch_prev_shift's
// v32), all h entries in one launch
hipError_t launch_prev_shift_hist(const Geo& g, const double* origin, int nrhs, const HistSrc& src,
                                  const Cx<double>* ainv_new, const WaveDev* wnew, Cx<float>* v32, size_t ve,
                                  hipStream_t st);
int gram_blocks(int Npad);
hipError_t launch_gram(int Npad, int nrhs, int h, const Cx<float>* W, const Cx<double>* b, double* partials,
                       hipStream_t st);
// The least-squares coefficients from the Gram partials, on the device (coef:
// [nrhs][HIST_MAX] complex)
hipError_t launch_proj_coef(int Npad, int nrhs, int h, const double* partials, Cx<double>* coef, hipStream_t st);
// x64 = sum_e coef[rhs][e] V[e] (coef: [nrhs][4] complex); esh = (1/alpha) x64
// and rf = b - sum_e coef[rhs][e] W[e] (FP32) where given.
hipError_t launch_hist_combine(const Geo& g, int nrhs, int h, const Cx<float>* V, const Cx<double>* coef,
                               Cx<double>* x64, const Cx<double>* ainv, Cx<float>* esh, const Cx<float>* W,
                               const Cx<double>* b, Cx<float>* rf, hipStream_t st);

// Raise a kernel's dynamic-LDS limit to the 160 KB of a gfx950 CU minus the
// kernel's static LDS (the attribute value is ignored beyond that).
inline hipError_t set_lds_limit(const void* fn, hipFuncAttribute attr, int lim) {
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    const int room = lim - (int)fa.sharedSizeBytes;
    return hipFuncSetAttribute(fn, attr, room);
}

// ---- compile-time specialised passes (kernels_ct.hip) ----
bool ct_supported(int n1, int n2, int n3);
template <class T>
int ct_available(int n, int tx);
template <class T>
bool ct_zpass_fits(int n, int tx, int zrb);
template <class T>
hipError_t launch_pass_ct(int which, int tx, int zrb, int ct, const Geo& g, const Tw<T>& tw, int nrhs,
                          const Cx<T>* x, Cx<T>* y, const Cx<T>* b, Cx<T>* slab, const Cx<T>* ghat, const Cx<T>* ainv,
                          const int* active, int mode, int dot, const Cx<T>* w, double* partials, const MvUpd& upd,
                          hipStream_t st);
hipError_t configure_ct_kernels();

// ---- learned initial guess (nn.hip) ----
struct dda_nn;
struct dda_wave_;  // the ABI's dda_wave
struct NnSiteView {
    long long uid;  // identifies the target's site list
    int n1, n2, n3, N, Npad, ncomp;
    const uint32_t* site_xyz;
    const uint8_t* site_comp;
    double origin[3];
    double kd;
    const double* m;  // 2 * ncomp
};
