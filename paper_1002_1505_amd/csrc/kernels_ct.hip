// Matvec passes specialised at compile time for cubic boxes n x n x n with
// n in {16, 32, 48, 64, 128}: the FFT length, radix plan, thread count and
// LDS layout are template constants.
//
//  * xy forward: as the generic pass (one block per plane and frequency
//    parity, scatter + 2D FFT in LDS).
//  * z pass: as the generic pass, tile width TX a template constant.
//  * xy inverse: one block per plane and *output* parity class (qx, qy).  The
//    n doubled-grid outputs x[2a + q] of an M = 2n point inverse DFT are an
//    n-point inverse DFT of Y_q[k] = conj(h[k])^q (X[k] + (-1)^q X[k + n])
//    evaluated at a < n/2, with h[k] = exp(-2 pi i k / M).  In 2D each class
//    pre-combines the four quadrants of the plane spectrum into an n x n LDS
//    plane, runs the inverse FFT along y on all columns and along x on the
//    first n/2 rows only, and gathers the sites (x, y) with x % 2 = qx and
//    y % 2 = qy, adding the diagonal term.  No accumulator crosses the FFTs.
//  * class-grouped slab (n = 64, specialised-kernel bit 8): the forward pass
//    stores the four quadrant partners (b, b + n/2 in y and in x) of each
//    parity block next to each other, slot (b'y n/2 + b'x) * 4 + 2 hy + hx;
//    the z pass, whose 16-column tiles then hold four whole partner groups,
//    replaces each group by its 2 x 2 Hadamard transform before the store, so
//    slot q of a group is already the class-q pre-combination and each
//    inverse block reads one value per frequency instead of four.  Within a
//    row the groups are ordered so that a tile holds two groups b'x and
//    n/2 - px - b'x whose columns fold onto the same tensor-spectrum
//    columns: a tile reads 8 spectrum columns instead of 16, and in a copy
//    of the spectrum with x columns in the same order they are adjacent.
#include <type_traits>

#include "dda_internal.h"

namespace {

__device__ __forceinline__ int fold_idx(int k, int n, int& sgn) {
    int f = k;
    sgn = 1;
    if (k > n) {
        f = 2 * n - k;
        sgn = -1;
    }
    return (f & 1) * (n / 2 + 1) + (f >> 1);
}

// Non-temporal store of a slab value: the 128^3 z pass's output, which at
// that size outgrows every cache before the inverse pass reads it and, stored
// normally, would push the tensor spectrum that a z-pass block reuses for
// every rhs out of the L2 (smaller slabs stay in the last-level cache between
// passes and are stored normally).
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_stream(Cx<float>* p, Cx<float> v) {
    f2v w;
    w.x = v.re;
    w.y = v.im;
    __builtin_nontemporal_store(w, reinterpret_cast<f2v*>(p));
}

// threads of the plane passes: 512 for n = 64 (8 waves per block; with 4
// blocks per CU by LDS that is 32 waves, against 16 with 256 threads and no
// room for 1024)
template <int N> constexpr int plane_threads() { return N >= 128 ? 1024 : (N == 64 ? 512 : 256); }
template <int N> constexpr int zpass_threads() { return N >= 128 ? 512 : 256; }

// UPD = 0: transform x.  UPD = 2: BiCGstab update s = r - alpha v, transform
// s and store it in pout (only the parity-0 block of a plane stores; pout
// never aliases an input).  alpha = rho / <rhat, v> is formed in the pass
// itself from the inverse pass's block partials of <rhat, v> (slot 0 of
// part, 12 n blocks per rhs).
struct UpdArgs {
    const void* r;
    const void* v;
    void* pout;
    BiState* st;
    const double* part;
};

// n = 64 and 128, FP32, class-grouped slab: one forward block per plane and
// x parity covers both y parities
template <class T, int N, bool G>
constexpr bool pfwd_pair() { return (N == 64 || N == 128) && G && sizeof(Cx<T>) == 8; }

// Store of a transformed plane of x parity px into the class-grouped slab
// (FP32): a group's four quadrant partners (y, x), (y, x + n/2),
// (y + n/2, x), (y + n/2, x + n/2) are 4 consecutive elements of the slab;
// lane l of a wave stores half l / 32 (rows y or y + n/2) of group l % 32 of
// the wave's 32 groups as one 16-byte store, so each store of the wave
// covers 1 KB without gaps.  The two halves of a group lie in one LDS bank,
// read by lanes of different half-waves.
template <int N, int NTH>
__device__ __forceinline__ void store_plane(Cx<float>* out, const Cx<float>* buf, int px, int tid) {
    constexpr int HN = N / 2, PITCH = N + 1;
    static_assert(NTH % 64 == 0, "whole waves");
    float4* o4 = reinterpret_cast<float4*>(out);
#pragma unroll 4
    for (int h = tid; h < N * N / 2; h += NTH) {
        const int gq = (h >> 6) * 32 + (h & 31), half = (h >> 5) & 1;
        const Cx<float>* q = buf + (gq / HN + half * HN) * PITCH + grp_bx(gq % HN, px, HN);
        const Cx<float> a0 = q[0], a1 = q[HN];
        o4[2 * (size_t)gq + half] = make_float4(a0.re, a0.im, a1.re, a1.im);
    }
}

template <class T, int N, int UPD, bool G>
__global__ void __launch_bounds__(plane_threads<N>()) k_pfwd_ct(const Cx<T>* __restrict__ x, Cx<T>* __restrict__ slab,
                                                                Geo g, Tw<T> tw, int nrhs, const int* __restrict__ active,
                                                                UpdArgs u) {
    constexpr int NTH = plane_threads<N>();
    constexpr int PITCH = N + 1;
    constexpr bool PAIR = pfwd_pair<T, N, G>();
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* t1 = reinterpret_cast<Cx<T>*>(smem_raw);
    Cx<T>* buf = t1 + N;
    const int nplanes = nrhs * 3 * N;
    const int b = blockIdx.x;
    // the blocks of a plane are 8 apart, so they run on one XCD and share
    // its L2 for the site values; PAIR: one block per x parity, both y
    // parities
    const int plane = PAIR ? ((b >> 3) >> 1) * 8 + (b & 7) : ((b >> 3) >> 2) * 8 + (b & 7);
    const int par = PAIR ? (b >> 3) & 1 : (b >> 3) & 3;
    // every scalar of the exit test is loaded before it (the rhs clamped into
    // range for blocks past the last plane; a site range is never reversed),
    // so the loads overlap instead of following one another
    const int rhs = min(plane / (3 * N), nrhs - 1);
    const int c = (plane / N) % 3, z = plane % N;
    const int j0 = g.plane_start[z], j1 = g.plane_start[z + 1];
    const int on = active ? active[rhs] : 1;
    if (plane >= nplanes || !on || j1 < j0) return;
    const int px = par & 1, py = par >> 1;
    const int tid = threadIdx.x;
    // gather operands: batches of UB sites per thread, every global load of a
    // batch issued (indices past the plane clamped to its last site, j1 > j0
    // here) before any is used; the first batch is issued now, so its latency
    // overlaps the set-up below
    constexpr int UB = 4;
    const size_t vo = ((size_t)rhs * 3 + c) * g.Npad;
    const Cx<T>* rv = reinterpret_cast<const Cx<T>*>(u.r);
    const Cx<T>* vv = reinterpret_cast<const Cx<T>*>(u.v);
    uint32_t sv[UB];
    Cx<T> xa[UB], xb[UB];
    auto load_batch = [&](int jb) {
#pragma unroll
        for (int k = 0; k < UB; ++k) {
            const int j = min(jb + k * NTH, j1 - 1);
            sv[k] = g.site_xyz[j];
            if (UPD == 0) {
                xa[k] = x[vo + j];
            } else {
                xa[k] = rv[vo + j];
                xb[k] = vv[vo + j];
            }
        }
    };
    if (j1 > j0) load_batch(j0 + tid);
    constexpr int NW = NTH / 64;
    __shared__ double red[2 * NW];
    if constexpr (UPD == 2) {
        // <rhat, v>: every block sums the 12 n block partials in one fixed
        // order (thread strides, wave totals, waves in order), so all blocks
        // of the pass hold the same alpha bit for bit
        constexpr int NB = 12 * N;
        const double* pp = u.part + (size_t)rhs * 4 * NB * 2;
        double ar = 0, ai = 0;
        for (int i = tid; i < NB; i += NTH) {
            ar += pp[2 * i];
            ai += pp[2 * i + 1];
        }
        ar = wave_total(ar);
        ai = wave_total(ai);
        if ((tid & 63) == 0) {
            red[2 * (tid >> 6)] = ar;
            red[2 * (tid >> 6) + 1] = ai;
        }
    }
    // the half-shift twiddles of the site coordinates next to the plane, so
    // the gather's lookups (addressed by the site just loaded) stay in LDS
    Cx<T>* th = buf + N * PITCH;
    for (int i = tid; i < N; i += NTH) {
        t1[i] = tw.f1[i];
        th[i] = tw.h1[i];
        th[N + i] = tw.h2[i];
    }
#pragma unroll 4
    for (int i = tid; i < N * PITCH; i += NTH) buf[i] = Cx<T>{0, 0};
    __syncthreads();
    Cx<T> c1 = {0, 0};
    if constexpr (UPD == 2) {
        double ar = 0, ai = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            ar += red[2 * w];
            ai += red[2 * w + 1];
        }
        // alpha = rho / <rhat, v>; a vanishing <rhat, v> (absolutely, or
        // against ||r||^2) gives alpha = 0 and marks a restart
        const double2 rho = make_double2(u.st[rhs].rho[0], u.st[rhs].rho[1]);
        const double an = sqrt(ar * ar + ai * ai);
        const int rs = (!(an > 1e-300) || !(an > 1e-14 * u.st[rhs].rr)) ? 1 : 0;
        const double2 al = rs ? make_double2(0.0, 0.0) : cdiv(rho, make_double2(ar, ai));
        c1 = Cx<T>{(T)al.x, (T)al.y};
        // the rhs's first block records alpha and the restart flag; no block
        // of this pass reads either field
        if (tid == 0 && par == 0 && plane % (3 * N) == 0) {
            u.st[rhs].alpha[0] = al.x;
            u.st[rhs].alpha[1] = al.y;
            u.st[rhs].restart = rs;
        }
    }
    Cx<T>* po = reinterpret_cast<Cx<T>*>(u.pout);
    for (int jb = j0 + tid; jb < j1; jb += UB * NTH) {
        if (jb != j0 + tid) load_batch(jb);
#pragma unroll
        for (int k = 0; k < UB; ++k) {
            const int j = jb + k * NTH;
            if (j < j1) {
                const int sx = sv[k] & 1023, sy = (sv[k] >> 10) & 1023;
                Cx<T> v;
                if (UPD == 0) {
                    v = xa[k];
                } else {
                    v = xa[k] - c1 * xb[k];
                    if (par == 0) po[vo + j] = v;
                }
                if (px) v = v * th[sx];
                if (py) v = v * th[N + sy];
                buf[sy * PITCH + sx] = v;
            }
        }
    }
    __syncthreads();
    ct_fft<T, -1, N, N, NTH, N, PITCH, 0, 1>(buf, t1, tid);   // along x: lines are rows
    if constexpr (PAIR) {
        // y parity 1 multiplies row y by h[y] before the transforms; that
        // factor is constant along a row, so it can be applied after the x
        // transform, which both y parities then share.  Each thread keeps
        // the elements (y, x) it restores: x = tid % N, y = tid / N + k NTH / N
        // These are also the rows that the first step (radix KR: 16 at
        // n = 128, 8 at n = 64) of the y transform combines for column x
        // (rows j + YS k, j = tid / N), so that step runs on the registers
        // and writes rows KR j + k, where the second and last step reads them.
        constexpr int KR = N * N / NTH, YS = NTH / N;
        static_assert(N * N % NTH == 0 && NTH % N == 0, "whole rows per thread step");
        static_assert(RadixPlan<N>::np == 2 && RadixPlan<N>::r[0] == KR && N / KR == YS,
                      "two steps, the first over the thread's rows");
        Cx<T> keep[KR];
#pragma unroll
        for (int k = 0; k < KR; ++k) keep[k] = buf[(tid / N + k * YS) * PITCH + tid % N];
        __syncthreads();
#pragma unroll
        for (int py = 0; py < 2; ++py) {
            Cx<T> t[KR];
#pragma unroll
            for (int k = 0; k < KR; ++k) t[k] = py ? keep[k] * th[N + tid / N + k * YS] : keep[k];
            bfly<T, -1, KR>(t);
#pragma unroll
            for (int k = 0; k < KR; ++k) buf[((tid / N) * KR + k) * PITCH + tid % N] = t[k];
            __syncthreads();
            ct_pass<T, -1, N, RadixPlan<N>::r[1], KR, N, NTH, N, 1, 0, PITCH>(buf, t1, tid);  // y, second step
            store_plane<N, NTH>(slab + ((((size_t)rhs * 3 + c) * N + z) * 4 + 2 * py + par) * (size_t)(N * N), buf,
                                px, tid);
            if (py == 0) __syncthreads();
        }
        return;
    }
    ct_fft<T, -1, N, N, NTH, N, 1, 0, PITCH>(buf, t1, tid);   // along y: lines are columns
    Cx<T>* out = slab + ((((size_t)rhs * 3 + c) * N + z) * 4 + par) * (size_t)(N * N);
    if constexpr (G && sizeof(Cx<T>) == 8) {
        store_plane<N, NTH>(out, buf, px, tid);
    } else if constexpr (G) {
        // one lane per group (FP64): its four quadrant partners lie in one
        // LDS bank, so the lane reads all four and stores them as 4
        // consecutive elements
        constexpr int HN = N / 2;
#pragma unroll 2
        for (int gq = tid; gq < N * N / 4; gq += NTH) {
            const Cx<T>* q = buf + (gq / HN) * PITCH + grp_bx(gq % HN, px, HN);
            const Cx<T> a0 = q[0], a1 = q[HN], a2 = q[HN * PITCH], a3 = q[HN * PITCH + HN];
            {
                Cx<T>* o = out + 4 * (size_t)gq;
                o[0] = a0;
                o[1] = a1;
                o[2] = a2;
                o[3] = a3;
            }
        }
    } else {
#pragma unroll 8
        for (int i = tid; i < N * N; i += NTH) out[i] = buf[(i / N) * PITCH + (i % N)];
    }
}

template <class T, int N, int TX>
__global__ void __launch_bounds__(zpass_threads<N>()) k_zpass_ct(Cx<T>* __restrict__ slab, const Cx<T>* __restrict__ gh,
                                                                 Geo g, Tw<T> tw, int nrhs, const int* __restrict__ active) {
    constexpr int NTH = zpass_threads<N>();
    constexpr int NCOL = 4 * N * N;
    constexpr int NTILE = NCOL / TX;
    constexpr int E = 3 * N * TX;
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* t3 = reinterpret_cast<Cx<T>*>(smem_raw);
    Cx<T>* W = t3 + N;
    const int rhs = blockIdx.x / NTILE, tile = blockIdx.x % NTILE;
    if (rhs >= nrhs) return;
    if (active && !active[rhs]) return;
    const int q0 = tile * TX;
    const int par = q0 / (N * N), rem = q0 % (N * N);
    const int px = par & 1, py = par >> 1;
    const int kyp = rem / N, kx0 = rem % N;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += NTH) t3[i] = tw.f3[i];
    Cx<T>* base = slab + (size_t)rhs * 3 * N * NCOL + q0;
    for (int e = tid; e < E; e += NTH) {
        const int col = e % TX, cz = e / TX;
        const int z = cz % N;
        const Cx<T> v = base[(size_t)cz * NCOL + col];
        W[e] = v;
        W[E + e] = v * tw.h3[z];
    }
    __syncthreads();
    ct_fft<T, -1, N, 6 * TX, NTH, TX, 1, N * TX, TX>(W, t3, tid);
    constexpr int H = N / 2 + 1;
    constexpr int D = 2 * H;
    constexpr size_t CS = (size_t)D * D * D;
    int sy;
    const int kyi = fold_idx(2 * kyp + py, N, sy);
    for (int i = tid; i < 2 * N * TX; i += NTH) {
        const int col = i % TX, zz = i / TX;
        const int kzp = zz % N, pz = zz / N;
        Cx<T>* w = W + pz * E;
        int sx, sz;
        const int kxi = fold_idx(2 * (kx0 + col) + px, N, sx);
        const int kzi = fold_idx(2 * kzp + pz, N, sz);
        const size_t gi = ((size_t)kzi * D + kyi) * D + kxi;
        const Cx<T> gxx = gh[gi], gxy = (T)(sx * sy) * gh[CS + gi], gxz = (T)(sx * sz) * gh[2 * CS + gi];
        const Cx<T> gyy = gh[3 * CS + gi], gyz = (T)(sy * sz) * gh[4 * CS + gi], gzz = gh[5 * CS + gi];
        const int o0 = kzp * TX + col, o1 = (N + kzp) * TX + col, o2 = (2 * N + kzp) * TX + col;
        const Cx<T> a0 = w[o0], a1 = w[o1], a2 = w[o2];
        w[o0] = gxx * a0 + gxy * a1 + gxz * a2;
        w[o1] = gxy * a0 + gyy * a1 + gyz * a2;
        w[o2] = gxz * a0 + gyz * a1 + gzz * a2;
    }
    __syncthreads();
    ct_fft<T, +1, N, 6 * TX, NTH, TX, 1, N * TX, TX>(W, t3, tid);
    for (int e = tid; e < E; e += NTH) {
        const int col = e % TX, cz = e / TX;
        const int z = cz % N;
        base[(size_t)cz * NCOL + col] = W[e] + cmulc(tw.h3[z], W[E + e]);
    }
}

// z pass over a tile of columns for up to RB right-hand sides per block.
// The tensor spectrum of the tile is loaded once into registers and reused
// for every right-hand side; each register entry serves the folded frequency
// kz_f in [0, n] and its mirror 2n - kz_f.
template <class T, int N, int TX, int RB>
__global__ void __launch_bounds__(zpass_threads<N>()) k_zpass2_ct(Cx<T>* __restrict__ slab,
                                                                  const Cx<T>* __restrict__ gh, Geo g, Tw<T> tw,
                                                                  int nrhs, const int* __restrict__ active) {
    constexpr int NTH = zpass_threads<N>();
    constexpr int NCOL = 4 * N * N;
    constexpr int E = 3 * N * TX;
    constexpr int NI = (N + 1) * TX;               // (folded kz, column) items
    constexpr int MI = (NI + NTH - 1) / NTH;       // items per thread
    constexpr int H = N / 2 + 1;
    constexpr int D = 2 * H;
    constexpr size_t CS = (size_t)D * D * D;
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* t3 = reinterpret_cast<Cx<T>*>(smem_raw);
    Cx<T>* W = t3 + N;
    const int tile = blockIdx.x;
    const int r0 = blockIdx.y * RB, r1 = min(nrhs, r0 + RB);
    bool any = false;
    for (int r = r0; r < r1; ++r) any |= (!active || active[r]);
    if (!any) return;
    const int q0 = tile * TX;
    const int par = q0 / (N * N), rem = q0 % (N * N);
    const int px = par & 1, py = par >> 1;
    const int kyp = rem / N, kx0 = rem % N;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += NTH) t3[i] = tw.f3[i];
    // spectrum of this tile in registers: 6 components per item
    Cx<T> G[MI][6];
    int sy;
    const int kyi = fold_idx(2 * kyp + py, N, sy);
#pragma unroll
    for (int m = 0; m < MI; ++m) {
        const int it = tid + m * NTH;
        if ((NI % NTH) == 0 || it < NI) {
            const int col = it % TX, kzf = it / TX;
            int sx, sz;
            const int kxi = fold_idx(2 * (kx0 + col) + px, N, sx);
            const int kzi = (kzf & 1) * H + (kzf >> 1);
            const size_t gi = ((size_t)kzi * D + kyi) * D + kxi;
#pragma unroll
            for (int q = 0; q < 6; ++q) G[m][q] = gh[q * CS + gi];
            G[m][1] = (T)(sx * sy) * G[m][1];
            G[m][2] = (T)sx * G[m][2];   // z sign applied per mirror below
            G[m][4] = (T)sy * G[m][4];
        }
    }
    for (int r = r0; r < r1; ++r) {
        if (active && !active[r]) continue;
        Cx<T>* base = slab + (size_t)r * 3 * N * NCOL + q0;
        for (int e = tid; e < E; e += NTH) {
            const int col = e % TX, cz = e / TX;
            const int z = cz % N;
            const Cx<T> v = base[(size_t)cz * NCOL + col];
            W[e] = v;
            W[E + e] = v * tw.h3[z];
        }
        __syncthreads();
        ct_fft<T, -1, N, 6 * TX, NTH, TX, 1, N * TX, TX>(W, t3, tid);
#pragma unroll
        for (int m = 0; m < MI; ++m) {
            const int it = tid + m * NTH;
            if ((NI % NTH) == 0 || it < NI) {
                const int col = it % TX, kzf = it / TX;
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    if (side == 1 && (kzf == 0 || kzf == N)) break;
                    const int kz = side ? 2 * N - kzf : kzf;
                    const T sz = side ? (T)-1 : (T)1;
                    Cx<T>* w = W + (kz & 1) * E;
                    const int kzp = kz >> 1;
                    const Cx<T> gxx = G[m][0], gxy = G[m][1], gxz = sz * G[m][2];
                    const Cx<T> gyy = G[m][3], gyz = sz * G[m][4], gzz = G[m][5];
                    const int o0 = kzp * TX + col, o1 = (N + kzp) * TX + col, o2 = (2 * N + kzp) * TX + col;
                    const Cx<T> a0 = w[o0], a1 = w[o1], a2 = w[o2];
                    w[o0] = gxx * a0 + gxy * a1 + gxz * a2;
                    w[o1] = gxy * a0 + gyy * a1 + gyz * a2;
                    w[o2] = gxz * a0 + gyz * a1 + gzz * a2;
                }
            }
        }
        __syncthreads();
        ct_fft<T, +1, N, 6 * TX, NTH, TX, 1, N * TX, TX>(W, t3, tid);
        for (int e = tid; e < E; e += NTH) {
            const int col = e % TX, cz = e / TX;
            const int z = cz % N;
            base[(size_t)cz * NCOL + col] = W[e] + cmulc(tw.h3[z], W[E + e]);
        }
        __syncthreads();
    }
}

// z pass as a two-factor decomposition N = 8 x 8 with the spectrum product
// in registers.  With z = z1 + 8 z2 and k = k2 + 8 k1, the forward N-point
// DFT is an 8-point DFT over z2 (thread (c, z1)), a twiddle w_N^(z1 k2), an
// exchange through LDS and an 8-point DFT over z1 (thread (c, k2)); the
// inverse runs the same steps backwards, so no digit reversal is needed and
// each direction crosses LDS once.  Thread (c, k2) multiplies the 3 vector
// components by the 3 x 3 tensor spectrum at kz = 2 k + pz for both
// frequency parities pz; the parity-1 input is pre-twiddled by h3 and its
// output post-twiddled by conj(h3).  One block per (tile of TX columns, rhs);
// block b runs on XCD b mod 8 and takes, in the order of that XCD's tile
// list, every rhs of one tile before the next tile, so that the tiles sharing
// tensor-spectrum columns read them from one L2.  gh is the spectrum with the
// 6 components of each frequency adjacent.
template <class T, int N, int TX>
__global__ void __launch_bounds__(TX * 8) k_zpass3_ct(Cx<T>* __restrict__ slab, const Cx<T>* __restrict__ gh,
                                                      Tw<T> tw, int nrhs, const int* __restrict__ active,
                                                      const int* __restrict__ tiles) {
    static_assert(N == 64, "two-factor z pass is written for N = 64");
    constexpr int R = 8;
    constexpr int NCOL = 4 * N * N;
    constexpr int H = N / 2 + 1;
    constexpr int D = 2 * H;
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* X = reinterpret_cast<Cx<T>*>(smem_raw);  // [a][k2][z1][c]
    constexpr int PER_XCD = 4 * N * N / TX / 8;
    const int b = blockIdx.x;
    const int pos = b >> 3;
    const int r = pos % nrhs;
    const int tile = tiles[(b & 7) * PER_XCD + pos / nrhs];
    // the tile index enters the exit test (it is never negative), so its load
    // is issued together with the flag's instead of after the branch
    if ((active && !active[r]) || tile < 0) return;
    const int tid = threadIdx.x;
    const int c = tid % TX, j = tid / TX;  // j: z1 in the outer steps, k2 in the inner ones
    const int q0 = tile * TX;
    const int par = q0 / (N * N), rem = q0 % (N * N);
    const int px = par & 1, py = par >> 1;
    const int kyp = rem / N, kx0 = rem % N;
    int sx, sy;
    const int kxi = fold_idx(2 * (kx0 + c) + px, N, sx);
    const int kyi = fold_idx(2 * kyp + py, N, sy);
    const T sxy = (T)(sx * sy);
    Cx<T> w[R];  // w_N^(j m)
#pragma unroll
    for (int m = 0; m < R; ++m) w[m] = tw.f3[j * m];
    // rhs base is uniform; per-thread offsets stay 32-bit (3 N NCOL < 2^32)
    Cx<T>* base = slab + (size_t)r * 3 * N * NCOL;
    const uint32_t o0 = (uint32_t)j * NCOL + q0 + c;
    Cx<T> acc[3][R];
#pragma unroll 1
    for (int pz = 0; pz < 2; ++pz) {
        // forward, outer factor: thread (c, z1 = j)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Cx<T> u[R];
#pragma unroll
            for (int z2 = 0; z2 < R; ++z2) u[z2] = base[o0 + (uint32_t)(a * N + R * z2) * NCOL];
            // pz is the loop counter (uniform): the twiddles load as one batch
            if (pz) {
                Cx<T> hz[R];
#pragma unroll
                for (int z2 = 0; z2 < R; ++z2) hz[z2] = tw.h3[j + R * z2];
#pragma unroll
                for (int z2 = 0; z2 < R; ++z2) u[z2] = u[z2] * hz[z2];
            }
            bfly<T, -1, R>(u);
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) X[((a * R + k2) * R + j) * TX + c] = k2 ? u[k2] * w[k2] : u[k2];
        }
        __syncthreads();
        // inner factor, tensor product, inverse inner factor: thread (c, k2 = j)
        {
            Cx<T> f[3][R];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
#pragma unroll
                for (int z1 = 0; z1 < R; ++z1) f[a][z1] = X[((a * R + j) * R + z1) * TX + c];
                bfly<T, -1, R>(f[a]);
            }
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) {
                // keep at most two frequencies of tensor loads in flight (register pressure)
                if (k1 % 2 == 0) __builtin_amdgcn_sched_barrier(0);
                const int kz = 2 * (j + R * k1) + pz;
                const bool mir = kz > N;
                const int kzf = mir ? 2 * N - kz : kz;
                const T sz = mir ? (T)-1 : (T)1;
                // spectrum with the 6 components of a frequency adjacent (48 or 96 bytes)
                const uint32_t gi = ((uint32_t)(pz * H + (kzf >> 1)) * D + kyi) * D + kxi;
                Cx<T> gg[6];
                if constexpr (sizeof(T) == 4) {
                    const float4* gp = reinterpret_cast<const float4*>(gh) + (size_t)gi * 3;
                    const float4 v0 = gp[0], v1 = gp[1], v2 = gp[2];
                    gg[0] = Cx<T>{v0.x, v0.y};
                    gg[1] = Cx<T>{v0.z, v0.w};
                    gg[2] = Cx<T>{v1.x, v1.y};
                    gg[3] = Cx<T>{v1.z, v1.w};
                    gg[4] = Cx<T>{v2.x, v2.y};
                    gg[5] = Cx<T>{v2.z, v2.w};
                } else {
#pragma unroll
                    for (int qq = 0; qq < 6; ++qq) gg[qq] = gh[(size_t)gi * 6 + qq];
                }
                const Cx<T> gxx = gg[0], gxy = sxy * gg[1], gxz = ((T)sx * sz) * gg[2];
                const Cx<T> gyy = gg[3], gyz = ((T)sy * sz) * gg[4], gzz = gg[5];
                const Cx<T> a0 = f[0][k1], a1 = f[1][k1], a2 = f[2][k1];
                f[0][k1] = gxx * a0 + gxy * a1 + gxz * a2;
                f[1][k1] = gxy * a0 + gyy * a1 + gyz * a2;
                f[2][k1] = gxz * a0 + gyz * a1 + gzz * a2;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                bfly<T, +1, R>(f[a]);
                // each thread rewrites exactly the slots it read above
#pragma unroll
                for (int z1 = 0; z1 < R; ++z1)
                    X[((a * R + j) * R + z1) * TX + c] = z1 ? cmulc(w[z1], f[a][z1]) : f[a][z1];
            }
        }
        __syncthreads();
        // inverse, outer factor: thread (c, z1 = j); the next parity's forward
        // step rewrites only these slots, so no barrier is needed before it
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Cx<T> u[R];
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) u[k2] = X[((a * R + k2) * R + j) * TX + c];
            bfly<T, +1, R>(u);
#pragma unroll
            for (int z2 = 0; z2 < R; ++z2) acc[a][z2] = pz ? acc[a][z2] + cmulc(tw.h3[j + R * z2], u[z2]) : u[z2];
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int z2 = 0; z2 < R; ++z2) base[o0 + (uint32_t)(a * N + R * z2) * NCOL] = acc[a][z2];
}

// The same two-factor z pass with the two frequency parities in the two
// halves of the block (threads pz * 8 TX + ...): each half runs its parity
// through its own LDS exchange buffer, and the parity-1 half hands its
// post-twiddled output to the parity-0 half through LDS.  Each thread then
// carries one parity's state, which halves the registers of the
// single-half version and raises the waves per SIMD.
//
// G: class-grouped slab.  Column c of a tile is quadrant partner (hy, hx) =
// (c >> 1 & 1, c & 1) of group c >> 2; the four partners of a group sit in
// one quad of lanes, which exchange values by DPP for the Hadamard step.
template <class T, int N, int TX, bool G>
__global__ void __launch_bounds__(TX * 16) k_zpass4_ct(Cx<T>* __restrict__ slab, const Cx<T>* __restrict__ gh,
                                                       Tw<T> tw, int nrhs, const int* __restrict__ active,
                                                       const int* __restrict__ tiles) {
    static_assert(N == 64, "two-factor z pass is written for N = 64");
    constexpr int R = 8;
    constexpr int NCOL = 4 * N * N;
    constexpr int H = N / 2 + 1;
    constexpr int D = 2 * H;
    constexpr int XS = 3 * N * TX;  // one exchange buffer [a][k2][z1][c]
    constexpr int PER_XCD = 4 * N * N / TX / 8;
    extern __shared__ unsigned char smem_raw[];
    const int b = blockIdx.x;
    const int pos = b >> 3;
    const int r = pos % nrhs;
    const int tile = tiles[(b & 7) * PER_XCD + pos / nrhs];
    // the tile index enters the exit test (it is never negative), so its load
    // is issued together with the flag's instead of after the branch
    if ((active && !active[r]) || tile < 0) return;
    const int tid = threadIdx.x;
    // each half is a whole number of waves, so the parity is wave-uniform;
    // saying so lets its branches below run on the scalar unit instead of
    // masking lanes, and the twiddle loads under them issue as one batch
    static_assert((TX * R) % 64 == 0, "halves of whole waves");
    const int pz = __builtin_amdgcn_readfirstlane(tid / (TX * R));
    const int tt = tid % (TX * R);
    const int c = tt % TX, j = tt / TX;  // j: z1 in the outer steps, k2 in the inner ones
    Cx<T>* X = reinterpret_cast<Cx<T>*>(smem_raw) + pz * XS;
    const int q0 = tile * TX;
    const int par = q0 / (N * N), rem = q0 % (N * N);
    const int px = par & 1, py = par >> 1;
    int sx, sy, kxi, kyi;
    if constexpr (G) {
        static_assert(TX % 4 == 0, "tiles of whole partner groups");
        constexpr int HN = N / 2;
        const int gq = (rem >> 2) + (c >> 2);
        // spectrum copy whose x columns follow the group order
        const int kx = 2 * (grp_bx(gq % HN, px, HN) + (c & 1) * HN) + px;
        const int fx = kx > N ? 2 * N - kx : kx;
        sx = kx > N ? -1 : 1;
        kxi = px * (HN + 1) + spec_xpos(fx >> 1, px, HN);
        kyi = fold_idx(2 * (gq / HN + ((c >> 1) & 1) * HN) + py, N, sy);
    } else {
        const int kyp = rem / N, kx0 = rem % N;
        kxi = fold_idx(2 * (kx0 + c) + px, N, sx);
        kyi = fold_idx(2 * kyp + py, N, sy);
    }
    const T sxy = (T)(sx * sy);
    Cx<T> w[R];  // w_N^(j m)
#pragma unroll
    for (int m = 0; m < R; ++m) w[m] = tw.f3[j * m];
    Cx<T>* base = slab + (size_t)r * 3 * N * NCOL;
    const uint32_t o0 = (uint32_t)j * NCOL + q0 + c;
    // half-shift twiddles of the parity-1 half (the same for all three components)
    Cx<T> h[R];
    if (pz) {
#pragma unroll
        for (int z2 = 0; z2 < R; ++z2) h[z2] = tw.h3[j + R * z2];
    }
    // forward, outer factor: thread (c, z1 = j) of half pz
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Cx<T> u[R];
#pragma unroll
        for (int z2 = 0; z2 < R; ++z2) u[z2] = base[o0 + (uint32_t)(a * N + R * z2) * NCOL];
        if (pz) {
#pragma unroll
            for (int z2 = 0; z2 < R; ++z2) u[z2] = u[z2] * h[z2];
        }
        bfly<T, -1, R>(u);
#pragma unroll
        for (int k2 = 0; k2 < R; ++k2) X[((a * R + k2) * R + j) * TX + c] = k2 ? u[k2] * w[k2] : u[k2];
    }
    // spectrum index of inner step k1 (frequency kz = 2 (j + 8 k1) + pz, folded)
    auto spec_at = [&](int k1) -> uint32_t {
        const int kz = 2 * (j + R * k1) + pz;
        const int kzf = kz > N ? 2 * N - kz : kz;
        return ((uint32_t)(pz * H + (kzf >> 1)) * D + kyi) * D + kxi;
    };
    // FP32: the first inner step's spectrum is loaded before the barrier, so
    // that its latency overlaps the wait (later steps load in turn: one step
    // ahead would cost a wave per SIMD in registers)
    float4 g0[3];
    if constexpr (sizeof(T) == 4) {
        const float4* gp = reinterpret_cast<const float4*>(gh) + (size_t)spec_at(0) * 3;
        g0[0] = gp[0];
        g0[1] = gp[1];
        g0[2] = gp[2];
    }
    __syncthreads();
    // inner factor, tensor product, inverse inner factor: thread (c, k2 = j)
    {
        Cx<T> f[3][R];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int z1 = 0; z1 < R; ++z1) f[a][z1] = X[((a * R + j) * R + z1) * TX + c];
            bfly<T, -1, R>(f[a]);
        }
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1) {
            const int kz = 2 * (j + R * k1) + pz;
            const T sz = kz > N ? (T)-1 : (T)1;
            const uint32_t gi = spec_at(k1);
            Cx<T> gg[6];
            if constexpr (sizeof(T) == 4) {
                const float4* gp = reinterpret_cast<const float4*>(gh) + (size_t)gi * 3;
                const float4 v0 = k1 ? gp[0] : g0[0], v1 = k1 ? gp[1] : g0[1], v2 = k1 ? gp[2] : g0[2];
                gg[0] = Cx<T>{v0.x, v0.y};
                gg[1] = Cx<T>{v0.z, v0.w};
                gg[2] = Cx<T>{v1.x, v1.y};
                gg[3] = Cx<T>{v1.z, v1.w};
                gg[4] = Cx<T>{v2.x, v2.y};
                gg[5] = Cx<T>{v2.z, v2.w};
            } else {
#pragma unroll
                for (int qq = 0; qq < 6; ++qq) gg[qq] = gh[(size_t)gi * 6 + qq];
            }
            const Cx<T> gxx = gg[0], gxy = sxy * gg[1], gxz = ((T)sx * sz) * gg[2];
            const Cx<T> gyy = gg[3], gyz = ((T)sy * sz) * gg[4], gzz = gg[5];
            const Cx<T> a0 = f[0][k1], a1 = f[1][k1], a2 = f[2][k1];
            f[0][k1] = gxx * a0 + gxy * a1 + gxz * a2;
            f[1][k1] = gxy * a0 + gyy * a1 + gyz * a2;
            f[2][k1] = gxz * a0 + gyz * a1 + gzz * a2;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            bfly<T, +1, R>(f[a]);
#pragma unroll
            for (int z1 = 0; z1 < R; ++z1)
                X[((a * R + j) * R + z1) * TX + c] = z1 ? cmulc(w[z1], f[a][z1]) : f[a][z1];
        }
    }
    __syncthreads();
    // inverse, outer factor: thread (c, z1 = j).  The parity-1 half writes its
    // post-twiddled output into the slots it has just read.
    Cx<T> u[3][R];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int k2 = 0; k2 < R; ++k2) u[a][k2] = X[((a * R + k2) * R + j) * TX + c];
        bfly<T, +1, R>(u[a]);
        if (pz)
#pragma unroll
            for (int z2 = 0; z2 < R; ++z2)
                X[((a * R + z2) * R + j) * TX + c] = cmulc(h[z2], u[a][z2]);
    }
    __syncthreads();
    if (pz) return;
    const Cx<T>* X1 = reinterpret_cast<const Cx<T>*>(smem_raw) + XS;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int z2 = 0; z2 < R; ++z2) {
            Cx<T> v = u[a][z2] + X1[((a * R + z2) * R + j) * TX + c];
            if constexpr (G) v = quad_hadamard(v, c);
            base[o0 + (uint32_t)(a * N + R * z2) * NCOL] = v;
        }
}

// m + s * (m of lane ^ 8 in the same row of 16 lanes), both parts: one
// v_fmac_f32 with a DPP row rotation by 8 per part (the compiler does not fold
// a DPP move into an FMAC).  The s_nop gives the two wait states between a
// VALU write of a register and a DPP read of it.  Every lane of the wave must
// be active.
__device__ __forceinline__ Cx<float> fma_row_xor8(Cx<float> m, float s) {
    Cx<float> d = m;
    asm("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %2, %4 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %3, %4 row_ror:8 row_mask:0xf bank_mask:0xf"
        : "+v"(d.re), "+v"(d.im)
        : "v"(m.re), "v"(m.im), "v"(s));
    return d;
}

// z pass of the n = 128 box (FP32) as a two-factor decomposition 128 = 16 x 8
// with one frequency parity per block half.  With z = z1 + 16 z2 and
// k = k2 + 8 k1, the forward DFT is an 8-point DFT over z2 (thread (c, z1),
// 16 threads per column), a twiddle w_128^(z1 k2), one exchange through LDS
// and a 16-point DFT over z1.  That 16-point DFT is split over a pair of
// lanes (8 apart in a row of 16): thread (c, k2, e) with e the parity of z1 takes
// the 8-point DFT over z1 = e + 2 z1' and the pair finishes it with one
// radix-2 step, F[k1' + 8 s] = G_0[k1'] + (-1)^s w_16^k1' G_1[k1'], lane e
// keeping s = e; so each thread holds 8 frequencies k = k2 + 8 k1' + 64 e of
// its column for the tensor product, the register load of the 64-point pass
// with twice the threads per column.  The inverse runs the same steps
// backwards; the outer threads apply both twiddles, so the inner steps need
// only the eight constants w_16^k1'.  The parity-1 half's shift h3[z] splits
// into a constant per z2 and a factor per z1 that joins the outer twiddles,
// so no twiddle beyond those eight per thread is held; that half hands its
// output to the parity-0 half through LDS.  Block b runs on XCD b mod 8 and
// takes one tile of its XCD's list for every rhs in turn.
//
// G: class-grouped slab, as in the n = 64 pass: a tile of 8 columns holds
// two partner groups (positions 2k, 2k + 1 of a row, whose columns fold onto
// the same spectrum columns), partner (hy, hx) = (c >> 1 & 1, c & 1) of
// group c >> 2 in lane c of a quad; the store replaces each group by its
// 2 x 2 Hadamard transform, and the spectrum copy's x columns follow the
// group order.
template <int TX, bool G>
__global__ void __launch_bounds__(TX * 32) __attribute__((amdgpu_waves_per_eu(3, 3))) k_zpass5_ct(Cx<float>* __restrict__ slab, const Cx<float>* __restrict__ gh,
                                                      Tw<float> tw, int nrhs, const int* __restrict__ active,
                                                      const int* __restrict__ tiles) {
    using T = float;
    constexpr int N = 128;
    constexpr int R2 = 8;   // outer factor: 8 points over z2
    constexpr int R1 = 16;  // inner factor: 16 points over z1 (radix 2 across a lane pair x 8)
    constexpr int NCOL = 4 * N * N;
    constexpr int H = N / 2 + 1;
    constexpr int D = 2 * H;
    constexpr int XS = 3 * R2 * R1 * TX;  // one exchange buffer [a][k2][z1][c]
    constexpr int PER_XCD = NCOL / TX / 8;
    static_assert(TX == 8, "lane layout: 8 columns, bit 3 of the lane is the parity of z1");
    static_assert(PER_XCD % 2 == 0, "whole tile pairs per XCD");
    extern __shared__ unsigned char smem_raw[];
    const int b = blockIdx.x;
    // block b takes tile list entry b / 8 of XCD b mod 8 and every rhs in
    // turn: the tile's spectrum columns, read again for each rhs within
    // microseconds by the same block, stay in the XCD's L2, and the twiddles
    // are loaded once.  Consecutive blocks of an XCD hold neighbouring tiles
    // (list entries 2i, 2i + 1, whose 64-byte row segments share 128-byte
    // lines) and walk the rhs in the same order.
    const int tile = tiles[(b & 7) * PER_XCD + (b >> 3)];
    if (tile < 0) return;
    const int tid = threadIdx.x;
    const int pz = __builtin_amdgcn_readfirstlane(tid / (TX * R1));
    const int tt = tid % (TX * R1);
    const int c = tt % TX, j = tt / TX;  // outer steps: j = z1; inner steps: j = 2 k2 + e
    Cx<T>* X = reinterpret_cast<Cx<T>*>(smem_raw) + pz * XS;
    // LDS slot of (a, k2, z1, c); bit 1 of z1 is flipped for odd k2, so the
    // inner steps' reads (four k2 and both e per wave) touch every bank pair
    // exactly twice, as the outer steps' accesses do
    auto xi = [c](int a, int k2, int z1) { return ((a * R2 + k2) * R1 + (z1 ^ ((k2 & 1) << 1))) * TX + c; };
    const int q0 = tile * TX;
    const int par = q0 / (N * N), rem = q0 % (N * N);
    const int px = par & 1, py = par >> 1;
    int sx, sy, kxi, kyi;
    if constexpr (G) {
        constexpr int HN = N / 2;
        const int gq = (rem >> 2) + (c >> 2);
        const int kx = 2 * (grp_bx(gq % HN, px, HN) + (c & 1) * HN) + px;
        const int fx = kx > N ? 2 * N - kx : kx;
        sx = kx > N ? -1 : 1;
        kxi = px * (HN + 1) + spec_xpos(fx >> 1, px, HN);
        kyi = fold_idx(2 * (gq / HN + ((c >> 1) & 1) * HN) + py, N, sy);
    } else {
        const int kyp = rem / N, kx0 = rem % N;
        kxi = fold_idx(2 * (kx0 + c) + px, N, sx);
        kyi = fold_idx(2 * kyp + py, N, sy);
    }
    const T sxy = (T)(sx * sy);
    const uint32_t o0_blk = (uint32_t)j * NCOL + q0 + c;
    // w_16^m = exp(-2 pi i m / 16), m < 8: the radix-2 twiddles of the inner
    // step and the z2-dependent part of the parity-1 half shift
    constexpr T C1 = (T)0.92387953251128675613, S1 = (T)0.38268343236508977173;
    constexpr T RS = (T)0.70710678118654752440;
    const Cx<T> w16[8] = {{1, 0}, {C1, -S1}, {RS, -RS}, {S1, -C1}, {0, -1}, {-S1, -C1}, {-RS, -RS}, {-C1, -S1}};
    // outer twiddles of thread z1 = j: w_128^(j k2) in the parity-0 half; in
    // the parity-1 half they absorb the common factor w_256^j of the half
    // shift h3[j + 16 z2] = w_256^j w_16^z2, giving w_256^(j (2 k2 + 1))
    // (from the h3 table, which holds w_256^q for q < 128, and
    // w_256^(q + 128) = -w_256^q); the factor w_16^z2 is a constant
    // held for the whole block in an LDS table WT[pz][m][z1] (thread tid
    // writes entry tid), read where they are applied
    Cx<T>* WT = reinterpret_cast<Cx<T>*>(smem_raw) + 2 * XS;
    static_assert(TX * 32 == 2 * R2 * R1, "one table entry per thread");
    {
        const int tpz = tid >> 7, tm = (tid >> 4) & (R2 - 1), tj = tid & (R1 - 1);
        const int q = tpz ? tj * (2 * tm + 1) : tj * tm;
        const Cx<T> hv = (tpz ? tw.h3 : tw.f3)[q & (N - 1)];
        WT[tid] = (q & N) ? Cx<T>{-hv.re, -hv.im} : hv;
    }
    const Cx<T>* w = WT + pz * R2 * R1 + j;  // w[m * R1]: factor m of thread z1 = j
    const int k2 = j >> 1, e = j & 1;
    const T sgn = e ? (T)-1 : (T)1, nsgn = -sgn;
    // w_16^m on lane e = 1 and 1 on lane e = 0 (a product with it replaces a
    // product followed by a per-lane select)
    const T fe = (T)e;
    auto wsel = [&](int m) -> Cx<T> { return Cx<T>{fmaf(fe, w16[m].re - (T)1, (T)1), fe * w16[m].im}; };
    // spectrum index of inner frequency k = k2 + 8 (k1' + 8 e), kz = 2 k + pz (folded)
    const uint32_t sp0_blk = (uint32_t)kyi * D + kxi;
    uint32_t sp0 = sp0_blk;
    auto spec_at = [&](int k1p) -> uint32_t {
        const int kz = 2 * (k2 + R2 * (k1p + 8 * e)) + pz;
        const int kzf = kz > N ? 2 * N - kz : kz;
        return (uint32_t)(pz * H + (kzf >> 1)) * (D * D) + sp0;
    };
    const Cx<T>* X1 = reinterpret_cast<const Cx<T>*>(smem_raw) + XS;
#pragma unroll 1
    for (int r = 0; r < nrhs; ++r) {
        if (active && !active[r]) continue;  // block-uniform
        Cx<T>* base = slab + (size_t)r * 3 * N * NCOL;
        // the lane offsets pass through an empty asm statement, so that the
        // addresses derived from them are formed inside the loop rather than
        // kept in registers across it
        uint32_t o0 = o0_blk;
        sp0 = sp0_blk;
        asm volatile("" : "+v"(o0), "+v"(sp0));
        // the twiddle table is written (first rhs), and the parity-1 half
        // rewrites the exchange buffer the parity-0 half read at the end of the
        // previous rhs
        __syncthreads();
        // forward, outer factor: thread (c, z1 = j)
    #pragma unroll
        for (int a = 0; a < 3; ++a) {
            Cx<T> u[R2];
    #pragma unroll
            for (int z2 = 0; z2 < R2; ++z2) u[z2] = base[o0 + (uint32_t)(a * N + R1 * z2) * NCOL];
            if (pz) {
    #pragma unroll
                for (int z2 = 1; z2 < R2; ++z2) u[z2] = w16[z2] * u[z2];
            }
            bfly<T, -1, R2>(u);
    #pragma unroll
            for (int k2o = 0; k2o < R2; ++k2o) X[xi(a, k2o, j)] = (k2o || pz) ? u[k2o] * w[k2o * R1] : u[k2o];
        }
        // the first frequency's spectrum is loaded before the barrier
        float4 g0[3];
        {
            const float4* gp = reinterpret_cast<const float4*>(gh) + (size_t)spec_at(0) * 3;
            g0[0] = gp[0];
            g0[1] = gp[1];
            g0[2] = gp[2];
        }
        __syncthreads();
        {
            Cx<T> f[3][R2];
    #pragma unroll
            for (int a = 0; a < 3; ++a) {
    #pragma unroll
                for (int z1p = 0; z1p < R2; ++z1p) f[a][z1p] = X[xi(a, k2, e + 2 * z1p)];
                bfly<T, -1, R2>(f[a]);
                // radix-2 step across the lane pair: lane e contributes G_0 or
                // w_16^k1' G_1 and keeps its own contribution + (-1)^e that of
                // its partner: F[k1'] on lane 0, -F[k1' + 8] on lane 1 (the
                // sign is carried through the tensor product, which is
                // linear, and taken back in the inverse step)
    #pragma unroll
                for (int k1p = 0; k1p < R2; ++k1p) {
                    if (k1p % 2 == 0) __builtin_amdgcn_sched_barrier(0);
                    const Cx<T> mine = k1p ? wsel(k1p) * f[a][k1p] : f[a][k1p];
                    f[a][k1p] = fma_row_xor8(mine, sgn);
                }
            }
    #pragma unroll
            for (int k1p = 0; k1p < R2; ++k1p) {
                // at most two frequencies of spectrum loads in flight (registers)
                if (k1p % 2 == 0) __builtin_amdgcn_sched_barrier(0);
                const int kz = 2 * (k2 + R2 * (k1p + 8 * e)) + pz;
                const T sz = kz > N ? (T)-1 : (T)1;
                const float4* gp = reinterpret_cast<const float4*>(gh) + (size_t)spec_at(k1p) * 3;
                const float4 v0 = k1p ? gp[0] : g0[0], v1 = k1p ? gp[1] : g0[1], v2 = k1p ? gp[2] : g0[2];
                const Cx<T> gxx = {v0.x, v0.y}, gxy = sxy * Cx<T>{v0.z, v0.w}, gxz = ((T)sx * sz) * Cx<T>{v1.x, v1.y};
                const Cx<T> gyy = {v1.z, v1.w}, gyz = ((T)sy * sz) * Cx<T>{v2.x, v2.y}, gzz = {v2.z, v2.w};
                const Cx<T> a0 = f[0][k1p], a1 = f[1][k1p], a2 = f[2][k1p];
                f[0][k1p] = gxx * a0 + gxy * a1 + gxz * a2;
                f[1][k1p] = gxy * a0 + gyy * a1 + gyz * a2;
                f[2][k1p] = gxz * a0 + gyz * a1 + gzz * a2;
            }
    #pragma unroll
            for (int a = 0; a < 3; ++a) {
                // inverse radix-2 step: lane e forms Y0 + Y1 (e = 0) or
                // (Y0 - Y1) conj(w_16^k1') (e = 1) from its value and its
                // partner's; lane 1 holds -Y1, so that is its own value
                // - (-1)^e times the partner's
    #pragma unroll
                for (int k1p = 0; k1p < R2; ++k1p) {
                    if (k1p % 2 == 0) __builtin_amdgcn_sched_barrier(0);
                    const Cx<T> s = fma_row_xor8(f[a][k1p], nsgn);
                    f[a][k1p] = k1p ? cmulc(wsel(k1p), s) : s;
                }
                bfly<T, +1, R2>(f[a]);
                // each thread rewrites exactly the slots it read above
    #pragma unroll
                for (int z1p = 0; z1p < R2; ++z1p) X[xi(a, k2, e + 2 * z1p)] = f[a][z1p];
            }
        }
        __syncthreads();
        // inverse, outer factor: thread (c, z1 = j), the conjugate twiddles; the
        // parity-1 half finishes its half shift with conj(w_16^z2) and writes its
        // output into the slots it has just read
        Cx<T> u[3][R2];
    #pragma unroll
        for (int a = 0; a < 3; ++a) {
    #pragma unroll
            for (int k2o = 0; k2o < R2; ++k2o) {
                const Cx<T> v = X[xi(a, k2o, j)];
                u[a][k2o] = (k2o || pz) ? cmulc(w[k2o * R1], v) : v;
            }
            bfly<T, +1, R2>(u[a]);
            if (pz) {
    #pragma unroll
                for (int z2 = 0; z2 < R2; ++z2) X[xi(a, z2, j)] = z2 ? cmulc(w16[z2], u[a][z2]) : u[a][z2];
            }
        }
        __syncthreads();
        if (!pz) {
    #pragma unroll
            for (int a = 0; a < 3; ++a)
    #pragma unroll
                for (int z2 = 0; z2 < R2; ++z2) {
                    Cx<T> v = u[a][z2] + X1[xi(a, z2, j)];
                    if constexpr (G) v = quad_hadamard(v, c);
                    st_stream(base + o0 + (uint32_t)(a * N + R1 * z2) * NCOL, v);
                }
        }
    }
}

template <int TX>
constexpr size_t zpass5_lds() { return (size_t)(2 * 3 * 8 * 16 * TX + 2 * 8 * 16) * sizeof(Cx<float>); }

// DOT = 1: per-block partial sums of conj(w_j) . y_j (slot 0); DOT = 2:
// conj(y_j) . x_j (slot 0) and |y_j|^2 (slot 1); DOT = 3: as DOT = 2 with
// |x_j|^2 in the imaginary part of slot 1, conj(w_j) . x_j (slot 2) and
// conj(w_j) . y_j (slot 3).  partials[rhs][slot][blk]
// with blk = (plane within rhs) * 4 + class, 12 n blocks per rhs.
template <class T, int N, int MODE, int DOT, bool G>
__global__ void __launch_bounds__(plane_threads<N>()) k_pinv_ct(const Cx<T>* __restrict__ slab, const Cx<T>* __restrict__ x,
                                                                Cx<T>* __restrict__ y, const Cx<T>* __restrict__ bvec,
                                                                const Cx<T>* __restrict__ ainv, Geo g, Tw<T> tw, int nrhs,
                                                                const int* __restrict__ active,
                                                                const Cx<T>* __restrict__ wv, double* __restrict__ partials) {
    constexpr int NTH = plane_threads<N>();
    constexpr int PITCH = N + 1;
    constexpr int NN = N * N;
    constexpr int HN = N / 2;
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* t1 = reinterpret_cast<Cx<T>*>(smem_raw);
    Cx<T>* buf = t1 + N;
    const int nplanes = nrhs * 3 * N;
    const int b = blockIdx.x;
    const int plane = ((b >> 3) >> 2) * 8 + (b & 7);
    const int q = (b >> 3) & 3;
    // every scalar of the exit test is loaded before it (the rhs clamped into
    // range for blocks past the last plane; a site range is never reversed),
    // so the loads overlap; the sites of output class q are stored
    // contiguously within the plane
    const int rhs = min(plane / (3 * N), nrhs - 1);
    const int c = (plane / N) % 3, z = plane % N;
    const int j0 = g.class_start[4 * z + q], j1 = g.class_start[4 * z + q + 1];
    const int on = active ? active[rhs] : 1;
    if (plane >= nplanes || !on || j1 < j0) return;
    const int qx = q & 1, qy = q >> 1;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += NTH) t1[i] = tw.f1[i];
    const Cx<T>* in = slab + (((size_t)rhs * 3 + c) * N + z) * 4 * (size_t)NN;
    const T sgx = qx ? (T)-1 : (T)1, sgy = qy ? (T)-1 : (T)1;
    constexpr int NI = NN / NTH;  // frequencies per thread
    // grouped slab with a two-step plan whose first radix is NI: a thread's
    // NI rows are the ones the first step of the y transform combines for
    // its column, so that step runs on its registers (see k_pinvq_ct)
    constexpr bool REG1 = G && NN % NTH == 0 && NTH % N == 0 && RadixPlan<N>::np == 2 &&
                          RadixPlan<N>::r[0] == NI && N / NI == NTH / N;
    if constexpr (G && NN % NTH == 0 && NTH % N == 0 && NI <= 16) {
        // grouped slab (one load per frequency): a thread keeps one column kx
        // (NTH is a multiple of n); all its loads are issued before the first
        // use, and the block-uniform class branches around the twiddles are
        // scalar.  Lanes run along the group positions of one frequency
        // parity px (t = px n/2 + position), so a load of the wave reads
        // consecutive groups of one class plane
        const int tpos = tid % N, px = tpos / HN, bx = grp_bx(tpos % HN, px, HN), kxp = 2 * bx + px;
        const int gs = (tpos % HN) * 4 + q;
        Cx<T> hy[NI];
        if (qy) {
#pragma unroll
            for (int i = 0; i < NI; ++i) hy[i] = tw.h2[(tid + i * NTH) / N];
        }
        const Cx<T> hx = qx ? tw.h1[kxp] : Cx<T>{1, 0};
        Cx<T> v[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int kyp = (tid + i * NTH) / N;
            const int by = kyp >> 1, py = kyp & 1;
            v[i] = in[(size_t)(py * 2 + px) * NN + by * HN * 4 + gs];
        }
        if (qx) {
#pragma unroll
            for (int i = 0; i < NI; ++i) v[i] = cmulc(hx, v[i]);
        }
        if (qy) {
#pragma unroll
            for (int i = 0; i < NI; ++i) v[i] = cmulc(hy[i], v[i]);
        }
        if constexpr (REG1) {
            bfly<T, +1, NI>(v);
#pragma unroll
            for (int i = 0; i < NI; ++i) buf[((tid / N) * NI + i) * PITCH + kxp] = v[i];
        } else {
#pragma unroll
            for (int i = 0; i < NI; ++i) buf[((tid + i * NTH) / N) * PITCH + kxp] = v[i];
        }
    } else if constexpr (!G && NN % NTH == 0 && NTH % N == 0) {
        // row layout (four quadrant loads per frequency): the same scheme in
        // batches of BI frequencies, which bounds the registers in flight
        constexpr int BI = NI < 4 ? NI : 4;
        static_assert(NI % BI == 0, "whole batches");
        const int kxp = tid % N, bx = kxp >> 1, px = kxp & 1;
        const Cx<T> hx = qx ? tw.h1[kxp] : Cx<T>{1, 0};
#pragma unroll 1
        for (int i0 = 0; i0 < NI; i0 += BI) {
            Cx<T> hy[BI], v[BI];
            if (qy) {
#pragma unroll
                for (int i = 0; i < BI; ++i) hy[i] = tw.h2[(tid + (i0 + i) * NTH) / N];
            }
#pragma unroll
            for (int i = 0; i < BI; ++i) {
                const int kyp = (tid + (i0 + i) * NTH) / N;
                const int by = kyp >> 1, py = kyp & 1;
                const Cx<T>* blk = in + (size_t)(py * 2 + px) * NN;
                const Cx<T> s00 = blk[by * N + bx], s10 = blk[by * N + bx + HN];
                const Cx<T> s01 = blk[(by + HN) * N + bx], s11 = blk[(by + HN) * N + bx + HN];
                v[i] = s00 + sgx * s10 + sgy * (s01 + sgx * s11);
            }
            if (qx) {
#pragma unroll
                for (int i = 0; i < BI; ++i) v[i] = cmulc(hx, v[i]);
            }
            if (qy) {
#pragma unroll
                for (int i = 0; i < BI; ++i) v[i] = cmulc(hy[i], v[i]);
            }
#pragma unroll
            for (int i = 0; i < BI; ++i) buf[((tid + (i0 + i) * NTH) / N) * PITCH + kxp] = v[i];
        }
    } else {
#pragma unroll 4
        for (int e = tid; e < NN; e += NTH) {
            const int kyp = e / N, kxp = e % N;
            const int bx = kxp >> 1, px = kxp & 1, by = kyp >> 1, py = kyp & 1;
            const Cx<T>* blk = in + (size_t)(py * 2 + px) * NN;
            Cx<T> v;
            if constexpr (G) {
                v = blk[(by * HN + grp_pos(bx, px, HN)) * 4 + q];
            } else {
                const Cx<T> s00 = blk[by * N + bx], s10 = blk[by * N + bx + HN];
                const Cx<T> s01 = blk[(by + HN) * N + bx], s11 = blk[(by + HN) * N + bx + HN];
                v = s00 + sgx * s10 + sgy * (s01 + sgx * s11);
            }
            if (qx) v = cmulc(tw.h1[kxp], v);
            if (qy) v = cmulc(tw.h2[kyp], v);
            buf[kyp * PITCH + kxp] = v;
        }
    }
    // the gather operands of the thread's first PF sites (site, composition,
    // x, and the rhs or dot-product vector) are requested before the
    // transforms, so that their latency overlaps them; the sites are visited
    // in the order j0 + tid, j0 + tid + NTH, ... either way
    constexpr int PF = 2;
    const size_t vo = ((size_t)rhs * 3 + c) * g.Npad;
    const Cx<T>* av = ainv + (size_t)rhs * g.ncomp;
    uint32_t pf_s[PF];
    int pf_c[PF];
    Cx<T> pf_x[PF], pf_w[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        // an index past the class is clamped into it (an empty class reads
        // site 0; neither value is used)
        const int j = j1 > j0 ? min(j0 + tid + k * NTH, j1 - 1) : 0;
        pf_s[k] = g.site_xyz[j];
        pf_c[k] = g.site_comp[j];
        pf_x[k] = x[vo + j];
        if (MODE == MV_RESID) pf_w[k] = bvec[vo + j];
        else if (DOT == 1 || DOT == 3) pf_w[k] = wv[vo + j];
    }
    __syncthreads();
    // only outputs below n/2 are read: rows y' < n/2 by the x transform,
    // columns x' < n/2 by the gather
    if constexpr (REG1)
        ct_pass<T, +1, N, RadixPlan<N>::r[1], NI, N, NTH, N, 1, 0, PITCH, HN>(buf, t1, tid);  // y, second step
    else
        ct_fft_keep<T, +1, N, N, NTH, N, 1, 0, PITCH, HN>(buf, t1, tid);  // along y, every column
    ct_fft_keep<T, +1, N, HN, NTH, HN, PITCH, 0, 1, HN>(buf, t1, tid);    // along x, rows y' < n/2
    double a0r = 0, a0i = 0, a1r = 0, a1i = 0, a2r = 0, a2i = 0, a3r = 0, a3i = 0;
    auto visit = [&](int j, uint32_t s, int cj, Cx<T> xj, Cx<T> wj) {
        const int sx = s & 1023, sy = (s >> 10) & 1023;
        Cx<T> v = buf[(sy >> 1) * PITCH + (sx >> 1)] + av[cj] * xj;
        if (MODE == MV_RESID) v = wj - v;
        y[vo + j] = v;
        if (DOT == 1) {
            a0r += (double)wj.re * v.re + (double)wj.im * v.im;
            a0i += (double)wj.re * v.im - (double)wj.im * v.re;
        } else if (DOT == 2 || DOT == 3) {
            a0r += (double)v.re * xj.re + (double)v.im * xj.im;
            a0i += (double)v.re * xj.im - (double)v.im * xj.re;
            a1r += (double)v.re * v.re + (double)v.im * v.im;
            if (DOT == 3) {
                a1i += (double)xj.re * xj.re + (double)xj.im * xj.im;
                a2r += (double)wj.re * xj.re + (double)wj.im * xj.im;
                a2i += (double)wj.re * xj.im - (double)wj.im * xj.re;
                a3r += (double)wj.re * v.re + (double)wj.im * v.im;
                a3i += (double)wj.re * v.im - (double)wj.im * v.re;
            }
        }
    };
#pragma unroll
    for (int k = 0; k < PF; ++k)
        if (j0 + tid + k * NTH < j1) visit(j0 + tid + k * NTH, pf_s[k], pf_c[k], pf_x[k], pf_w[k]);
#pragma unroll 2
    for (int j = j0 + tid + PF * NTH; j < j1; j += NTH) {
        Cx<T> wj = {0, 0};
        if (MODE == MV_RESID) wj = bvec[vo + j];
        else if (DOT == 1 || DOT == 3) wj = wv[vo + j];
        visit(j, g.site_xyz[j], g.site_comp[j], x[vo + j], wj);
    }
    if (DOT) {
        __shared__ double sh[8 * 16];
        const int nblk = 12 * N;
        const int blk = (plane % (3 * N)) * 4 + q;
        double red[8] = {a0r, a0i, a1r, a1i, a2r, a2i, a3r, a3i};
        block_sum_n<DOT == 3 ? 8 : (DOT == 2 ? 3 : 2)>(red, sh);
        const double s0r = red[0], s0i = red[1];
        const double s1r = DOT >= 2 ? red[2] : 0, s1i = DOT == 3 ? red[3] : 0;
        const double s2r = DOT == 3 ? red[4] : 0, s2i = DOT == 3 ? red[5] : 0;
        const double s3r = DOT == 3 ? red[6] : 0, s3i = DOT == 3 ? red[7] : 0;
        if (tid == 0) {
            double* o = partials + ((size_t)rhs * 4 * nblk + blk) * 2;
            o[0] = s0r;
            o[1] = s0i;
            if (DOT >= 2) {
                o[2 * nblk] = s1r;
                o[2 * nblk + 1] = s1i;
            }
            if (DOT == 3) {
                o[4 * nblk] = s2r;
                o[4 * nblk + 1] = s2i;
                o[6 * nblk] = s3r;
                o[6 * nblk + 1] = s3i;
            }
        }
    }
}

// Inverse plane pass for n = 128, FP32, class-grouped slab: one block per
// output class q and four consecutive planes z0 .. z0 + 3 (same rhs and
// component) runs them in turn, as k_pinv_ct runs one plane.  The plane
// fills the LDS, so one block runs per CU and nothing else hides a block's
// slab loads; here the loads of the next plane are issued right after the
// current plane's values are in LDS and arrive while it is transformed and
// gathered.  The four class blocks of a plane group are 8 apart, so they run
// on one XCD at about the same time and share the L2 lines of the grouped
// slab (a 128-byte line holds four groups' values of all four classes).
// Partial sums are written per plane and class, as k_pinv_ct writes them.
template <int MODE, int DOT>
__global__ void __launch_bounds__(1024) k_pinvq_ct(const Cx<float>* __restrict__ slab, const Cx<float>* __restrict__ x,
                                                   Cx<float>* __restrict__ y, const Cx<float>* __restrict__ bvec,
                                                   const Cx<float>* __restrict__ ainv, Geo g, Tw<float> tw, int nrhs,
                                                   const int* __restrict__ active, const Cx<float>* __restrict__ wv,
                                                   double* __restrict__ partials) {
    using T = float;
    constexpr int N = 128, NTH = 1024, PITCH = N + 1, NN = N * N, HN = N / 2, NI = NN / NTH, YS = NTH / N;
    static_assert(NTH == plane_threads<N>() && NN % NTH == 0 && NTH % N == 0, "thread layout");
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* t1 = reinterpret_cast<Cx<T>*>(smem_raw);
    Cx<T>* buf = t1 + N;
    Cx<T>* th = buf + N * PITCH;  // half-shift twiddles: x at [0, n), y at [n, 2n)
    constexpr int NP = 4;  // planes per block
    static_assert(N % NP == 0, "plane groups within one rhs and component");
    const int nplanes = nrhs * 3 * N;
    const int b = blockIdx.x;
    const int q = (b >> 3) & 3;
    const int plane0 = ((b >> 5) * 8 + (b & 7)) * NP;
    const int rhs = min(plane0 / (3 * N), nrhs - 1);
    const int c = (plane0 / N) % 3, z0 = plane0 % N;
    const int on = active ? active[rhs] : 1;
    if (plane0 >= nplanes || !on) return;
    const int qx = q & 1, qy = q >> 1;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += NTH) {
        t1[i] = tw.f1[i];
        th[i] = tw.h1[i];
        th[N + i] = tw.h2[i];
    }
    const Cx<T>* in = slab + (((size_t)rhs * 3 + c) * N + z0) * 4 * (size_t)NN;
    // a thread keeps one column kx for every plane; lanes run along the group
    // positions of one frequency parity px, so a load of the wave reads
    // consecutive groups of one class plane
    const int tpos = tid % N, px = tpos / HN, bx = grp_bx(tpos % HN, px, HN), kxp = 2 * bx + px;
    // frequency row kyp = tid / n + i YS of element i: its parity is the
    // thread's own (YS is even), so element i lies i (YS / 2) group rows
    // past element 0 in the same parity-block plane.  The loads are buffer
    // loads over the group's planes: one 32-bit byte offset of the thread
    // plus a block-uniform offset (plane and element) in a scalar register,
    // so no per-element address stays live across the transforms.  The
    // buffer's extent is the NP planes' four parity blocks each, which
    // bounds every load (an offset past it reads zero).  The last descriptor
    // word selects 32-bit data for raw (untyped) loads on this chip family.
    static_assert(YS % 2 == 0, "one y parity per thread");
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<Cx<T>*>(in), (short)0, (int)(NP * 4 * NN * sizeof(Cx<T>)), 0x00020000);
    const int boff = (((tid / N) & 1) * 2 + px) * NN * (int)sizeof(Cx<T>) +
                     (((tid / N) >> 1) * HN * 4 + (tpos % HN) * 4) * (int)sizeof(Cx<T>);
    Cx<T> v[NI];
    auto load_plane = [&](int kp) {
#pragma unroll
        for (int i = 0; i < NI; ++i)
            v[i] = __builtin_bit_cast(Cx<T>, __builtin_amdgcn_raw_buffer_load_b64(
                                                 rs, boff, (kp * 4 * NN + q + i * (YS / 2) * HN * 4) * (int)sizeof(Cx<T>), 0));
    };
    load_plane(0);
    const size_t vo = ((size_t)rhs * 3 + c) * g.Npad;
    const Cx<T>* av = ainv + (size_t)rhs * g.ncomp;
    __syncthreads();
#pragma unroll 1
    for (int kp = 0; kp < NP; ++kp) {
        // the thread index passes through an empty asm statement, so the
        // transforms' index arithmetic is redone per plane instead of being
        // hoisted out of the loop and held in registers across it
        int ltid = tid;
        asm volatile("" : "+v"(ltid));
        const int z = z0 + kp, plane = plane0 + kp;
        const int j0 = g.class_start[4 * z + q], j1 = g.class_start[4 * z + q + 1];
        {
            // the first radix-16 step of the y transform runs on the
            // registers: the thread's NI values are the rows kyp = j + YS i
            // (j = tid / n) of its column, which that step combines; its
            // outputs go to rows NI j + i, where the transform's second step
            // reads them
            static_assert(RadixPlan<N>::r[0] == NI && N / NI == YS, "first step over the thread's rows");
            const Cx<T> hx = th[kxp];
            Cx<T> t[NI];
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                const int kyp = tid / N + i * YS;
                t[i] = v[i];
                if (qx) t[i] = cmulc(hx, t[i]);
                if (qy) t[i] = cmulc(th[N + kyp], t[i]);
            }
            bfly<T, +1, NI>(t);
#pragma unroll
            for (int i = 0; i < NI; ++i) buf[((tid / N) * NI + i) * PITCH + kxp] = t[i];
        }
        // gather operands of the thread's first PF sites, then the next
        // plane's slab values
        constexpr int PF = 2;
        uint32_t pf_s[PF];
        int pf_c[PF];
        Cx<T> pf_x[PF], pf_w[PF];
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int j = j1 > j0 ? min(j0 + ltid + k * NTH, j1 - 1) : 0;
            pf_s[k] = g.site_xyz[j];
            pf_c[k] = g.site_comp[j];
            pf_x[k] = x[vo + j];
            if (MODE == MV_RESID) pf_w[k] = bvec[vo + j];
            else if (DOT == 1 || DOT == 3) pf_w[k] = wv[vo + j];
        }
        if (kp + 1 < NP) load_plane(kp + 1);
        __syncthreads();
        // only outputs below n/2 are read: rows y' < n/2 by the x
        // transform, columns x' < n/2 by the gather
        static_assert(RadixPlan<N>::np == 2, "two steps");
        ct_pass<T, +1, N, RadixPlan<N>::r[1], NI, N, NTH, N, 1, 0, PITCH, HN>(buf, t1, ltid);  // y, second step
        ct_fft_keep<T, +1, N, HN, NTH, HN, PITCH, 0, 1, HN>(buf, t1, ltid);  // along x, rows y' < n/2
        double a0r = 0, a0i = 0, a1r = 0, a1i = 0, a2r = 0, a2i = 0, a3r = 0, a3i = 0;
        auto visit = [&](int j, uint32_t s, int cj, Cx<T> xj, Cx<T> wj) {
            const int sx = s & 1023, sy = (s >> 10) & 1023;
            Cx<T> val = buf[(sy >> 1) * PITCH + (sx >> 1)] + av[cj] * xj;
            if (MODE == MV_RESID) val = wj - val;
            y[vo + j] = val;
            if (DOT == 1) {
                a0r += (double)wj.re * val.re + (double)wj.im * val.im;
                a0i += (double)wj.re * val.im - (double)wj.im * val.re;
            } else if (DOT == 2 || DOT == 3) {
                a0r += (double)val.re * xj.re + (double)val.im * xj.im;
                a0i += (double)val.re * xj.im - (double)val.im * xj.re;
                a1r += (double)val.re * val.re + (double)val.im * val.im;
                if (DOT == 3) {
                    a1i += (double)xj.re * xj.re + (double)xj.im * xj.im;
                    a2r += (double)wj.re * xj.re + (double)wj.im * xj.im;
                    a2i += (double)wj.re * xj.im - (double)wj.im * xj.re;
                    a3r += (double)wj.re * val.re + (double)wj.im * val.im;
                    a3i += (double)wj.re * val.im - (double)wj.im * val.re;
                }
            }
        };
#pragma unroll
        for (int k = 0; k < PF; ++k)
            if (j0 + ltid + k * NTH < j1) visit(j0 + ltid + k * NTH, pf_s[k], pf_c[k], pf_x[k], pf_w[k]);
#pragma unroll 2
        for (int j = j0 + ltid + PF * NTH; j < j1; j += NTH) {
            Cx<T> wj = {0, 0};
            if (MODE == MV_RESID) wj = bvec[vo + j];
            else if (DOT == 1 || DOT == 3) wj = wv[vo + j];
            visit(j, g.site_xyz[j], g.site_comp[j], x[vo + j], wj);
        }
        if (DOT) {
            __shared__ double sh[8 * 16];
            const int nblk = 12 * N;
            const int blk = (plane % (3 * N)) * 4 + q;
            double red[8] = {a0r, a0i, a1r, a1i, a2r, a2i, a3r, a3i};
            block_sum_n<DOT == 3 ? 8 : (DOT == 2 ? 3 : 2)>(red, sh);
            if (ltid == 0) {
                double* o = partials + ((size_t)rhs * 4 * nblk + blk) * 2;
                o[0] = red[0];
                o[1] = red[1];
                if (DOT >= 2) {
                    o[2 * nblk] = red[2];
                    o[2 * nblk + 1] = DOT == 3 ? red[3] : 0;
                }
                if (DOT == 3) {
                    o[4 * nblk] = red[4];
                    o[4 * nblk + 1] = red[5];
                    o[6 * nblk] = red[6];
                    o[6 * nblk + 1] = red[7];
                }
            }
        }
        // every read of the plane (and of the partial-sum scratch) ends
        // before the next plane is written
        __syncthreads();
    }
}

// Inverse plane pass for n = 64 as two-factor 8 x 8 transforms with one LDS
// exchange per axis.  Block per (plane, output parity class q) as above; the
// class pre-combination of the four quadrants feeds registers directly.
// Along y (all 64 columns): with ky = m1 + 8 m2 and y' = n2 + 8 n1, thread
// (kx, m1) does the 8-point transform over m2 and the twiddle w^(-m1 n2),
// thread (kx, n2) the transform over m1; only y' < n/2 is kept.  Along x on
// those 32 rows the same two steps keep x' < n/2.  LDS: rows of the first
// exchange [n2][m1][kx], then the 32 kept rows (pitch n + 1), the second
// exchange [n2][m1][y'] and the 32 x 32 result (pitch n/2 + 1).
template <class T, int N, int MODE, int DOT, bool G>
__global__ void __launch_bounds__(256) k_pinv3_ct(const Cx<T>* __restrict__ slab, const Cx<T>* __restrict__ x,
                                                  Cx<T>* __restrict__ y, const Cx<T>* __restrict__ bvec,
                                                  const Cx<T>* __restrict__ ainv, Geo g, Tw<T> tw, int nrhs,
                                                  const int* __restrict__ active, const Cx<T>* __restrict__ wv,
                                                  double* __restrict__ partials) {
    static_assert(N == 64, "two-factor plane pass is written for n = 64");
    constexpr int R = 8, NN = N * N, HN = N / 2;
    constexpr int PY = N + 1;       // pitch of the kept rows
    constexpr int X2OFF = HN * PY;  // second exchange after the kept rows
    constexpr int PF = HN + 1;      // pitch of the result
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* S = reinterpret_cast<Cx<T>*>(smem_raw);
    const int nplanes = nrhs * 3 * N;
    const int b = blockIdx.x;
    const int plane = ((b >> 3) >> 2) * 8 + (b & 7);
    const int q = (b >> 3) & 3;
    if (plane >= nplanes) return;
    const int rhs = plane / (3 * N);
    if (active && !active[rhs]) return;
    const int c = (plane / N) % 3, z = plane % N;
    const int qx = q & 1, qy = q >> 1;
    const int tid = threadIdx.x;
    const Cx<T>* in = slab + (((size_t)rhs * 3 + c) * N + z) * 4 * (size_t)NN;
    const T sgx = qx ? (T)-1 : (T)1, sgy = qy ? (T)-1 : (T)1;
    // y, outer factor: thread (kx, m1) for m1 in {g, g + 4}
    {
        const int kx = tid & (N - 1), g4 = tid >> 6;
        const int bx = kx >> 1, px = kx & 1;
        const Cx<T> hx = tw.h1[kx];
        // slot of this thread's column in a row of the grouped slab
        const int gs = G ? grp_pos(bx, px, HN) * 4 + q : 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int m1 = g4 + 4 * h;
            // ky = m1 + 8 m2 keeps the parity of m1: one quadrant block per h
            const Cx<T>* blk = in + (size_t)((m1 & 1) * 2 + px) * NN;
            // the class is block-uniform, so these branches are scalar and
            // every load of the step is in flight before the first use
            Cx<T> hy[R];
            if (qy) {
#pragma unroll
                for (int m2 = 0; m2 < R; ++m2) hy[m2] = tw.h2[m1 + R * m2];
            }
            Cx<T> u[R];
#pragma unroll
            for (int m2 = 0; m2 < R; ++m2) {
                const int by = (m1 + R * m2) >> 1;
                if constexpr (G) {
                    u[m2] = blk[by * HN * 4 + gs];
                } else {
                    const Cx<T> s00 = blk[by * N + bx], s10 = blk[by * N + bx + HN];
                    const Cx<T> s01 = blk[(by + HN) * N + bx], s11 = blk[(by + HN) * N + bx + HN];
                    u[m2] = s00 + sgx * s10 + sgy * (s01 + sgx * s11);
                }
            }
            if (qx) {
#pragma unroll
                for (int m2 = 0; m2 < R; ++m2) u[m2] = cmulc(hx, u[m2]);
            }
            if (qy) {
#pragma unroll
                for (int m2 = 0; m2 < R; ++m2) u[m2] = cmulc(hy[m2], u[m2]);
            }
            bfly<T, +1, R>(u);
#pragma unroll
            for (int n2 = 0; n2 < R; ++n2) S[(n2 * R + m1) * N + kx] = n2 ? cmulc(tw.f1[m1 * n2], u[n2]) : u[n2];
        }
    }
    __syncthreads();
    // y, inner factor: thread (kx, n2) for n2 in {g, g + 4}; keep y' = n2 + 8 n1 < n/2
    {
        const int kx = tid & (N - 1), g4 = tid >> 6;
        Cx<T> o[2][R];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int n2 = g4 + 4 * h;
#pragma unroll
            for (int m1 = 0; m1 < R; ++m1) o[h][m1] = S[(n2 * R + m1) * N + kx];
            bfly<T, +1, R>(o[h]);
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int n1 = 0; n1 < R / 2; ++n1) S[(g4 + 4 * h + R * n1) * PY + kx] = o[h][n1];
    }
    __syncthreads();
    // x on the kept rows, outer factor: thread (y', m1) with y' fastest
    {
        const int yr = tid & (HN - 1), m1 = tid >> 5;
        Cx<T> u[R];
#pragma unroll
        for (int m2 = 0; m2 < R; ++m2) u[m2] = S[yr * PY + m1 + R * m2];
        bfly<T, +1, R>(u);
#pragma unroll
        for (int n2 = 0; n2 < R; ++n2)
            S[X2OFF + (n2 * R + m1) * HN + yr] = n2 ? cmulc(tw.f1[m1 * n2], u[n2]) : u[n2];
    }
    __syncthreads();
    // x, inner factor: thread (y', n2); keep x' = n2 + 8 n1 < n/2; the result
    // overwrites the kept rows, which are no longer read
    {
        const int yr = tid & (HN - 1), n2 = tid >> 5;
        Cx<T> o[R];
#pragma unroll
        for (int m1 = 0; m1 < R; ++m1) o[m1] = S[X2OFF + (n2 * R + m1) * HN + yr];
        bfly<T, +1, R>(o);
#pragma unroll
        for (int n1 = 0; n1 < R / 2; ++n1) S[yr * PF + n2 + R * n1] = o[n1];
    }
    __syncthreads();
    const size_t vo = ((size_t)rhs * 3 + c) * g.Npad;
    const Cx<T>* av = ainv + (size_t)rhs * g.ncomp;
    // the sites of output class q are stored contiguously within the plane
    const int j0 = g.class_start[4 * z + q], j1 = g.class_start[4 * z + q + 1];
    double a0r = 0, a0i = 0, a1r = 0, a1i = 0, a2r = 0, a2i = 0, a3r = 0, a3i = 0;
#pragma unroll 2
    for (int j = j0 + tid; j < j1; j += 256) {
        const uint32_t s = g.site_xyz[j];
        const int sx = s & 1023, sy = (s >> 10) & 1023;
        const Cx<T> xj = x[vo + j];
        Cx<T> v = S[(sy >> 1) * PF + (sx >> 1)] + av[g.site_comp[j]] * xj;
        if (MODE == MV_RESID) v = bvec[vo + j] - v;
        y[vo + j] = v;
        if (DOT == 1) {
            const Cx<T> wj = wv[vo + j];
            a0r += (double)wj.re * v.re + (double)wj.im * v.im;
            a0i += (double)wj.re * v.im - (double)wj.im * v.re;
        } else if (DOT == 2 || DOT == 3) {
            a0r += (double)v.re * xj.re + (double)v.im * xj.im;
            a0i += (double)v.re * xj.im - (double)v.im * xj.re;
            a1r += (double)v.re * v.re + (double)v.im * v.im;
            if (DOT == 3) {
                const Cx<T> wj = wv[vo + j];
                a1i += (double)xj.re * xj.re + (double)xj.im * xj.im;
                a2r += (double)wj.re * xj.re + (double)wj.im * xj.im;
                a2i += (double)wj.re * xj.im - (double)wj.im * xj.re;
                a3r += (double)wj.re * v.re + (double)wj.im * v.im;
                a3i += (double)wj.re * v.im - (double)wj.im * v.re;
            }
        }
    }
    if (DOT) {
        __shared__ double sh[8 * 16];
        const int nblk = 12 * N;
        const int blk = (plane % (3 * N)) * 4 + q;
        double red[8] = {a0r, a0i, a1r, a1i, a2r, a2i, a3r, a3i};
        block_sum_n<DOT == 3 ? 8 : (DOT == 2 ? 3 : 2)>(red, sh);
        const double s0r = red[0], s0i = red[1];
        const double s1r = DOT >= 2 ? red[2] : 0, s1i = DOT == 3 ? red[3] : 0;
        const double s2r = DOT == 3 ? red[4] : 0, s2i = DOT == 3 ? red[5] : 0;
        const double s3r = DOT == 3 ? red[6] : 0, s3i = DOT == 3 ? red[7] : 0;
        if (tid == 0) {
            double* o = partials + ((size_t)rhs * 4 * nblk + blk) * 2;
            o[0] = s0r;
            o[1] = s0i;
            if (DOT >= 2) {
                o[2 * nblk] = s1r;
                o[2 * nblk + 1] = s1i;
            }
            if (DOT == 3) {
                o[4 * nblk] = s2r;
                o[4 * nblk + 1] = s2i;
                o[6 * nblk] = s3r;
                o[6 * nblk + 1] = s3i;
            }
        }
    }
}

template <class T, int N>
constexpr size_t plane_lds() { return (size_t)(3 * N + N * (N + 1)) * sizeof(Cx<T>); }
template <class T, int N, int TX>
constexpr size_t zpass_lds() { return (size_t)(N + 6 * N * TX) * sizeof(Cx<T>); }
template <class T, int N, int TX>
constexpr size_t zpass3_lds() { return (size_t)3 * N * TX * sizeof(Cx<T>); }
template <class T, int N, int TX>
constexpr size_t zpass4_lds() { return (size_t)2 * 3 * N * TX * sizeof(Cx<T>); }
constexpr size_t LDS_MAX = 160 * 1024;

template <class T, int N, int MODE, int DOT, bool G>
void launch_pinv_g(int nblk, bool two_factor, const Geo& g, const Tw<T>& tw, int nrhs, const Cx<T>* x, Cx<T>* y,
                   const Cx<T>* b, const Cx<T>* slab, const Cx<T>* ainv, const int* active, const Cx<T>* w,
                   double* partials, hipStream_t st) {
    if constexpr (N == 128 && G && std::is_same<T, float>::value) {
        // one block per class and group of 4 planes (nplanes is a multiple
        // of 4), in groups of 8 blocks
        const int ngrp = nrhs * 3 * N / 4;
        hipLaunchKernelGGL((k_pinvq_ct<MODE, DOT>), dim3((ngrp + 7) / 8 * 8 * 4), dim3(plane_threads<N>()),
                           (plane_lds<T, N>()), st,
                           slab, x, y, b, ainv, g, tw, nrhs, active, w, partials);
        return;
    }
    if constexpr (N == 64) {
        if (two_factor) {
            hipLaunchKernelGGL((k_pinv3_ct<T, N, MODE, DOT, G>), dim3(nblk), dim3(256), (plane_lds<T, N>()), st, slab,
                               x, y, b, ainv, g, tw, nrhs, active, w, partials);
            return;
        }
    }
    hipLaunchKernelGGL((k_pinv_ct<T, N, MODE, DOT, G>), dim3(nblk), dim3(plane_threads<N>()), (plane_lds<T, N>()), st,
                       slab, x, y, b, ainv, g, tw, nrhs, active, w, partials);
}

// grouped: class-grouped slab (n = 64 and 128)
template <class T, int N, int MODE, int DOT>
void launch_pinv(int nblk, bool two_factor, bool grouped, const Geo& g, const Tw<T>& tw, int nrhs, const Cx<T>* x,
                 Cx<T>* y, const Cx<T>* b, const Cx<T>* slab, const Cx<T>* ainv, const int* active, const Cx<T>* w,
                 double* partials, hipStream_t st) {
    if constexpr (N == 64 || N == 128)
        if (grouped)
            return launch_pinv_g<T, N, MODE, DOT, true>(nblk, two_factor, g, tw, nrhs, x, y, b, slab, ainv, active, w,
                                                        partials, st);
    launch_pinv_g<T, N, MODE, DOT, false>(nblk, two_factor, g, tw, nrhs, x, y, b, slab, ainv, active, w, partials, st);
}

template <class T, int N, int UPD>
void launch_pfwd(int nblk, bool grouped, const Geo& g, const Tw<T>& tw, int nrhs, const Cx<T>* x, Cx<T>* slab,
                 const int* active, const UpdArgs& ua, hipStream_t st) {
    if constexpr (N == 64 || N == 128) {
        if (grouped) {
            // nblk counts 4 blocks per 8-plane group member; a paired block
            // covers two of them
            if constexpr (pfwd_pair<T, N, true>()) nblk /= 2;
            hipLaunchKernelGGL((k_pfwd_ct<T, N, UPD, true>), dim3(nblk), dim3(plane_threads<N>()), (plane_lds<T, N>()),
                               st, x, slab, g, tw, nrhs, active, ua);
            return;
        }
    }
    hipLaunchKernelGGL((k_pfwd_ct<T, N, UPD, false>), dim3(nblk), dim3(plane_threads<N>()), (plane_lds<T, N>()), st,
                       x, slab, g, tw, nrhs, active, ua);
}

template <class T, int N>
hipError_t pass_n(int which, int tx, int zrb, int ct, const Geo& g, const Tw<T>& tw, int nrhs, const Cx<T>* x, Cx<T>* y,
                  const Cx<T>* b, Cx<T>* slab, const Cx<T>* ghat, const Cx<T>* ainv, const int* active, int mode,
                  int dot, const Cx<T>* w, double* partials, const MvUpd& upd, hipStream_t st) {
    const int nplanes = nrhs * 3 * N;
    const int nblk_plane = (nplanes + 7) / 8 * 8 * 4;
    if (which == 2 && !x) return hipErrorInvalidValue;        // diagonal term reads x
    if (which == 0 && upd.mode == 0 && !x) return hipErrorInvalidValue;
    if (which == 0 || which == 2) {
        if constexpr (plane_lds<T, N>() > LDS_MAX) {
            return hipErrorNotSupported;
        } else {
            const bool tf = (ct & 4) != 0, gr = (ct & 8) != 0;
            if (which == 0) {
                const UpdArgs ua{upd.r, upd.v, upd.pout, upd.st, upd.part};
                if (upd.mode == 2) launch_pfwd<T, N, 2>(nblk_plane, gr, g, tw, nrhs, x, slab, active, ua, st);
                else if (upd.mode == 0) launch_pfwd<T, N, 0>(nblk_plane, gr, g, tw, nrhs, x, slab, active, ua, st);
                else return hipErrorInvalidValue;
            } else if (mode == MV_AX) {
                if (dot == 1) launch_pinv<T, N, MV_AX, 1>(nblk_plane, tf, gr, g, tw, nrhs, x, y, b, slab, ainv, active, w, partials, st);
                else if (dot == 2) launch_pinv<T, N, MV_AX, 2>(nblk_plane, tf, gr, g, tw, nrhs, x, y, b, slab, ainv, active, w, partials, st);
                else if (dot == 3) launch_pinv<T, N, MV_AX, 3>(nblk_plane, tf, gr, g, tw, nrhs, x, y, b, slab, ainv, active, w, partials, st);
                else launch_pinv<T, N, MV_AX, 0>(nblk_plane, tf, gr, g, tw, nrhs, x, y, b, slab, ainv, active, w, partials, st);
            } else {
                launch_pinv<T, N, MV_RESID, 0>(nblk_plane, tf, gr, g, tw, nrhs, x, y, b, slab, ainv, active, w, partials, st);
            }
            return hipGetLastError();
        }
    }
    const int ntile = 4 * N * N;
    if (zrb == 4) {
        if constexpr (N != 128 || !std::is_same<T, float>::value) {
            return hipErrorNotSupported;
        } else {
            const int* tl = (ct & 8) ? g.ztiles8g : g.ztiles8;
            if (tx != 8 || !tl) return hipErrorNotSupported;
            if (ct & 8)
                hipLaunchKernelGGL((k_zpass5_ct<8, true>), dim3(ntile / 8), dim3(8 * 32), (zpass5_lds<8>()), st, slab,
                                   ghat, tw, nrhs, active, tl);
            else
                hipLaunchKernelGGL((k_zpass5_ct<8, false>), dim3(ntile / 8), dim3(8 * 32), (zpass5_lds<8>()), st, slab,
                                   ghat, tw, nrhs, active, tl);
            return hipGetLastError();
        }
    }
    if (zrb == 3) {
        if constexpr (N != 64) {
            return hipErrorNotSupported;
        } else {
            const int* tl = (ct & 8) ? g.ztiles16g : g.ztiles16;
            if (tx != 16 || !tl) return hipErrorNotSupported;
            if constexpr (zpass4_lds<T, N, 16>() > LDS_MAX) {
                return hipErrorNotSupported;
            } else {
                if (ct & 8)
                    hipLaunchKernelGGL((k_zpass4_ct<T, N, 16, true>), dim3(nrhs * (ntile / 16)), dim3(16 * 16),
                                       (zpass4_lds<T, N, 16>()), st, slab, ghat, tw, nrhs, active, tl);
                else
                    hipLaunchKernelGGL((k_zpass4_ct<T, N, 16, false>), dim3(nrhs * (ntile / 16)), dim3(16 * 16),
                                       (zpass4_lds<T, N, 16>()), st, slab, ghat, tw, nrhs, active, tl);
                return hipGetLastError();
            }
        }
    }
    if (zrb == 2) {
        if constexpr (N != 64) {
            return hipErrorNotSupported;
        } else {
#define ZP3(TXV)                                                                                                   \
    if (tx == TXV) {                                                                                               \
        if constexpr (zpass3_lds<T, N, TXV>() > LDS_MAX) {                                                         \
            return hipErrorNotSupported;                                                                           \
        } else {                                                                                                   \
            const int* tl = TXV == 16 ? g.ztiles16 : g.ztiles32;                                               \
            if (!tl) return hipErrorNotSupported;                                                              \
            hipLaunchKernelGGL((k_zpass3_ct<T, N, TXV>), dim3(nrhs * (ntile / TXV)), dim3(TXV * 8),               \
                               (zpass3_lds<T, N, TXV>()), st, slab, ghat, tw, nrhs, active, tl);                    \
            return hipGetLastError();                                                                              \
        }                                                                                                          \
    }
            ZP3(16)
            ZP3(32)
#undef ZP3
            return hipErrorNotSupported;
        }
    }
#define ZP2(TXV)                                                                                                   \
    if (tx == TXV && zrb == 1) {                                                                                   \
        if constexpr (zpass_lds<T, N, TXV>() > LDS_MAX || (N % TXV) != 0) {                                        \
            return hipErrorNotSupported;                                                                           \
        } else {                                                                                                   \
            hipLaunchKernelGGL((k_zpass2_ct<T, N, TXV, 8>), dim3(ntile / TXV, (nrhs + 7) / 8),                     \
                               dim3(zpass_threads<N>()), (zpass_lds<T, N, TXV>()), st, slab, ghat, g, tw, nrhs,    \
                               active);                                                                            \
            return hipGetLastError();                                                                              \
        }                                                                                                          \
    }
    ZP2(8)
    ZP2(16)
    ZP2(32)
#undef ZP2
#define ZP(TXV)                                                                                                    \
    if (tx == TXV) {                                                                                               \
        if constexpr (zpass_lds<T, N, TXV>() > LDS_MAX || (N % TXV) != 0) {                                        \
            return hipErrorNotSupported;                                                                           \
        } else {                                                                                                   \
            hipLaunchKernelGGL((k_zpass_ct<T, N, TXV>), dim3(nrhs * (ntile / TXV)), dim3(zpass_threads<N>()),      \
                               (zpass_lds<T, N, TXV>()), st, slab, ghat, g, tw, nrhs, active);                      \
            return hipGetLastError();                                                                              \
        }                                                                                                          \
    }
    ZP(8)
    ZP(16)
    ZP(32)
#undef ZP
    return hipErrorNotSupported;
}

template <class T, int N>
hipError_t set_attrs_n() {
    const int lim = 160 * 1024;
    hipError_t e = hipSuccess;
    if constexpr (plane_lds<T, N>() <= LDS_MAX) {
        const void* fns[] = {(const void*)k_pfwd_ct<T, N, 0, false>, (const void*)k_pfwd_ct<T, N, 2, false>,
                             (const void*)k_pinv_ct<T, N, MV_AX, 0, false>, (const void*)k_pinv_ct<T, N, MV_AX, 1, false>,
                             (const void*)k_pinv_ct<T, N, MV_AX, 2, false>, (const void*)k_pinv_ct<T, N, MV_AX, 3, false>,
                             (const void*)k_pinv_ct<T, N, MV_RESID, 0, false>};
        for (const void* f : fns)
            if (e == hipSuccess) e = set_lds_limit(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if constexpr (N == 64) {
            const void* f3[] = {
                (const void*)k_pinv3_ct<T, N, MV_AX, 0, false>, (const void*)k_pinv3_ct<T, N, MV_AX, 1, false>,
                (const void*)k_pinv3_ct<T, N, MV_AX, 2, false>, (const void*)k_pinv3_ct<T, N, MV_AX, 3, false>,
                (const void*)k_pinv3_ct<T, N, MV_RESID, 0, false>,
                (const void*)k_pfwd_ct<T, N, 0, true>, (const void*)k_pfwd_ct<T, N, 2, true>,
                (const void*)k_pinv_ct<T, N, MV_AX, 0, true>, (const void*)k_pinv_ct<T, N, MV_AX, 1, true>,
                (const void*)k_pinv_ct<T, N, MV_AX, 2, true>, (const void*)k_pinv_ct<T, N, MV_AX, 3, true>,
                (const void*)k_pinv_ct<T, N, MV_RESID, 0, true>,
                (const void*)k_pinv3_ct<T, N, MV_AX, 0, true>, (const void*)k_pinv3_ct<T, N, MV_AX, 1, true>,
                (const void*)k_pinv3_ct<T, N, MV_AX, 2, true>, (const void*)k_pinv3_ct<T, N, MV_AX, 3, true>,
                (const void*)k_pinv3_ct<T, N, MV_RESID, 0, true>};
            for (const void* f : f3)
                if (e == hipSuccess) e = set_lds_limit(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        }
        if constexpr (N == 128) {
            const void* fg[] = {
                (const void*)k_pfwd_ct<T, N, 0, true>, (const void*)k_pfwd_ct<T, N, 2, true>,
                (const void*)k_pinv_ct<T, N, MV_AX, 0, true>, (const void*)k_pinv_ct<T, N, MV_AX, 1, true>,
                (const void*)k_pinv_ct<T, N, MV_AX, 2, true>, (const void*)k_pinv_ct<T, N, MV_AX, 3, true>,
                (const void*)k_pinv_ct<T, N, MV_RESID, 0, true>};
            for (const void* f : fg)
                if (e == hipSuccess) e = set_lds_limit(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
            if constexpr (std::is_same<T, float>::value) {
                const void* fq[] = {(const void*)k_pinvq_ct<MV_AX, 0>, (const void*)k_pinvq_ct<MV_AX, 1>,
                                    (const void*)k_pinvq_ct<MV_AX, 2>, (const void*)k_pinvq_ct<MV_AX, 3>,
                                    (const void*)k_pinvq_ct<MV_RESID, 0>};
                for (const void* f : fq)
                    if (e == hipSuccess) e = set_lds_limit(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
            }
        }
    }
    if constexpr (zpass_lds<T, N, 8>() <= LDS_MAX && N % 8 == 0) {
        if (e == hipSuccess)
            e = set_lds_limit((const void*)k_zpass_ct<T, N, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e == hipSuccess)
            e = set_lds_limit((const void*)k_zpass2_ct<T, N, 8, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    }
    if constexpr (zpass_lds<T, N, 16>() <= LDS_MAX && N % 16 == 0) {
        if (e == hipSuccess)
            e = set_lds_limit((const void*)k_zpass_ct<T, N, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e == hipSuccess)
            e = set_lds_limit((const void*)k_zpass2_ct<T, N, 16, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    }
    if constexpr (zpass_lds<T, N, 32>() <= LDS_MAX && N % 32 == 0) {
        if (e == hipSuccess)
            e = set_lds_limit((const void*)k_zpass_ct<T, N, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e == hipSuccess)
            e = set_lds_limit((const void*)k_zpass2_ct<T, N, 32, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    }
    if constexpr (N == 128 && std::is_same<T, float>::value) {
        if (e == hipSuccess)
            e = set_lds_limit((const void*)k_zpass5_ct<8, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e == hipSuccess)
            e = set_lds_limit((const void*)k_zpass5_ct<8, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    }
    if constexpr (N == 64) {
        if (e == hipSuccess)
            e = set_lds_limit((const void*)k_zpass4_ct<T, N, 16, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e == hipSuccess)
            e = set_lds_limit((const void*)k_zpass4_ct<T, N, 16, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e == hipSuccess)
            e = set_lds_limit((const void*)k_zpass3_ct<T, N, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if constexpr (zpass3_lds<T, N, 32>() <= LDS_MAX)
            if (e == hipSuccess)
                e = set_lds_limit((const void*)k_zpass3_ct<T, N, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    }
    return e;
}

}  // namespace

bool ct_supported(int n1, int n2, int n3) {
    if (n1 != n2 || n2 != n3) return false;
    return n1 == 16 || n1 == 32 || n1 == 48 || n1 == 64 || n1 == 128;
}

template <class T>
hipError_t launch_pass_ct(int which, int tx, int zrb, int ct, const Geo& g, const Tw<T>& tw, int nrhs,
                          const Cx<T>* x, Cx<T>* y, const Cx<T>* b, Cx<T>* slab, const Cx<T>* ghat, const Cx<T>* ainv,
                          const int* active, int mode, int dot, const Cx<T>* w, double* partials, const MvUpd& upd,
                          hipStream_t st) {
    if (!ct_supported(g.n1, g.n2, g.n3)) return hipErrorNotSupported;
#define PN(NV) pass_n<T, NV>(which, tx, zrb, ct, g, tw, nrhs, x, y, b, slab, ghat, ainv, active, mode, dot, w, partials, upd, st)
    switch (g.n1) {
        case 16: return PN(16);
        case 32: return PN(32);
        case 48: return PN(48);
        case 64: return PN(64);
        default: return PN(128);
    }
#undef PN
}

template <class T>
bool ct_zpass_fits(int n, int tx, int zrb);

// Which passes of a cubic box of side n have a specialised kernel in precision
// T with z tile tx: bit 0 planes, bit 1 z pass, bit 2 two-factor inverse
// plane pass, bit 3 class-grouped slab (with z pass variants 3 and 4 only).
template <class T>
int ct_available(int n, int tx) {
    auto planes = [](size_t lds) { return lds <= LDS_MAX; };
    int bits = 0;
    if (!ct_supported(n, n, n)) return 0;
    if (planes((size_t)(3 * n + n * (n + 1)) * sizeof(Cx<T>))) bits |= 1;  // as plane_lds
    if ((bits & 1) && n == 64) bits |= 4;  // two-factor inverse plane pass
    if (ct_zpass_fits<T>(n, tx, 0) || ct_zpass_fits<T>(n, tx, 2) || ct_zpass_fits<T>(n, tx, 4)) bits |= 2;
    if ((bits & 3) == 3 && (ct_zpass_fits<T>(n, tx, 3) || ct_zpass_fits<T>(n, tx, 4))) bits |= 8;  // class-grouped slab
    return bits;
}

// Whether z-pass variant zrb (0, 1: LDS lines; 2: two-factor, n = 64) has a
// kernel for a cubic box of side n with z tile tx in precision T.
template <class T>
bool ct_zpass_fits(int n, int tx, int zrb) {
    if (!ct_supported(n, n, n) || !(tx == 8 || tx == 16 || tx == 32) || n % tx) return false;
    if (zrb == 2) return n == 64 && tx >= 16 && (size_t)3 * n * tx * sizeof(Cx<T>) <= LDS_MAX;
    if (zrb == 3) return n == 64 && tx == 16 && (size_t)6 * n * tx * sizeof(Cx<T>) <= LDS_MAX;
    if (zrb == 4) return n == 128 && tx == 8 && std::is_same<T, float>::value;
    return (zrb == 0 || zrb == 1) && (size_t)(n + 6 * n * tx) * sizeof(Cx<T>) <= LDS_MAX;
}

hipError_t configure_ct_kernels() {
    hipError_t e;
#define A(T, N) \
    if ((e = set_attrs_n<T, N>()) != hipSuccess) return e;
    A(float, 16) A(float, 32) A(float, 48) A(float, 64) A(float, 128)
    A(double, 16) A(double, 32) A(double, 48) A(double, 64) A(double, 128)
#undef A
    return hipSuccess;
}

template hipError_t launch_pass_ct<float>(int, int, int, int, const Geo&, const Tw<float>&, int, const Cx<float>*,
                                          Cx<float>*, const Cx<float>*, Cx<float>*, const Cx<float>*, const Cx<float>*,
                                          const int*, int, int, const Cx<float>*, double*, const MvUpd&, hipStream_t);
template hipError_t launch_pass_ct<double>(int, int, int, int, const Geo&, const Tw<double>&, int, const Cx<double>*,
                                           Cx<double>*, const Cx<double>*, Cx<double>*, const Cx<double>*,
                                           const Cx<double>*, const int*, int, int, const Cx<double>*, double*,
                                           const MvUpd&, hipStream_t);
template int ct_available<float>(int, int);
template int ct_available<double>(int, int);
template bool ct_zpass_fits<float>(int, int, int);
template bool ct_zpass_fits<double>(int, int, int);
