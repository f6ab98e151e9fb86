// Device-side building blocks of the DDA solver for gfx950: complex arithmetic,
// radix-2/3/4/5/8 butterflies and an in-LDS Stockham FFT over batches of lines.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

template <class T>
struct alignas(2 * sizeof(T)) Cx {
    T re, im;
};

template <class T> __host__ __device__ __forceinline__ Cx<T> mk(T a, T b) { return Cx<T>{a, b}; }
template <class T> __host__ __device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __host__ __device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __host__ __device__ __forceinline__ Cx<T> operator*(Cx<T> a, Cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> __host__ __device__ __forceinline__ Cx<T> operator*(T s, Cx<T> a) { return {s * a.re, s * a.im}; }
template <class T> __host__ __device__ __forceinline__ Cx<T> conj(Cx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <class T> __host__ __device__ __forceinline__ Cx<T> cmulc(Cx<T> a, Cx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// a * (s i), s = +1 or -1
template <class T, int S> __device__ __forceinline__ Cx<T> mul_si(Cx<T> a) {
    return S > 0 ? Cx<T>{-a.im, a.re} : Cx<T>{a.im, -a.re};
}
template <class To, class Ti> __device__ __forceinline__ Cx<To> cvt(Cx<Ti> a) { return {(To)a.re, (To)a.im}; }

// Value held by lane (lane ^ M) of the same group of four lanes, M in {1, 2}:
// a DPP quad permutation, no LDS round trip.  Every lane of the wave must be
// active.
template <int M> __device__ __forceinline__ int quad_xor_i(int v) {
    static_assert(M == 1 || M == 2, "quad lanes 1 or 2 apart");
    return __builtin_amdgcn_mov_dpp(v, M == 1 ? 0xB1 : 0x4E, 0xF, 0xF, false);
}
template <int M> __device__ __forceinline__ float quad_xor(float v) { return __int_as_float(quad_xor_i<M>(__float_as_int(v))); }
template <int M> __device__ __forceinline__ double quad_xor(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)quad_xor_i<M>((int)(unsigned)b), hi = (unsigned)quad_xor_i<M>((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int M, class T> __device__ __forceinline__ Cx<T> quad_xor(Cx<T> v) {
    return {quad_xor<M>(v.re), quad_xor<M>(v.im)};
}
// Class-grouped slab of the n = 64 matvec: group position p in a row of
// H = n/2 groups holds b'x = grp_bx(p, px), frequency parity px.  The folded
// spectrum column of b'x + n/2 is that of H - px - b'x, so positions
// (2k, 2k + 1) hold such a pair: (k, H - 1 - k) for px = 1; (k + 1, H - k - 1)
// for px = 0, where b'x = 0 and b'x = H/2 fold onto themselves and take the
// last two places.  grp_pos is the inverse.
// Both are select chains (no early returns), so a lane-dependent argument
// costs a few conditional moves rather than divergent branches.
__device__ __forceinline__ int grp_bx(int p, int px, int H) {
    const int k = p >> 1, odd = p & 1;
    const int b1 = odd ? H - 1 - k : k;
    const int b0 = p < H - 2 ? (odd ? H - 1 - k : k + 1) : (p == H - 2 ? 0 : H / 2);
    return px ? b1 : b0;
}
__device__ __forceinline__ int grp_pos(int b, int px, int H) {
    const bool lo = b < H / 2;
    const int p1 = lo ? 2 * b : 2 * (H - 1 - b) + 1;
    const int p0 = b == 0 ? H - 2 : (b == H / 2 ? H - 1 : (lo ? 2 * (b - 1) : 2 * (H - b - 1) + 1));
    return px ? p1 : p0;
}
// Slot of folded column f/2 = u (0..H) of parity half px in the spectrum copy
// that follows the group order (u = H, the even half's Nyquist column and the
// odd half's unused slot, stays last).
__device__ __forceinline__ int spec_xpos(int u, int px, int H) { return u == H ? H : grp_pos(u, px, H); }

// 2 x 2 Hadamard transform over the four lanes of a quad, lane bits (hy, hx):
// lane (qy, qx) returns sum over (hy, hx) of (-1)^(qx hx + qy hy) v(hy, hx).
template <class T> __device__ __forceinline__ Cx<T> quad_hadamard(Cx<T> v, int lane) {
    // lane bit set: partner minus own value, else own plus partner, as
    // o + s v with s = -1 or +1 (one rounding either way, the same bits)
    const T s1 = (lane & 1) ? (T)-1 : (T)1, s2 = (lane & 2) ? (T)-1 : (T)1;
    Cx<T> o = quad_xor<1>(v);
    v = Cx<T>{s1 * v.re + o.re, s1 * v.im + o.im};
    o = quad_xor<2>(v);
    return Cx<T>{s2 * v.re + o.re, s2 * v.im + o.im};
}

// ---------------------------------------------------------------------------
// Butterflies: DFT of length R in registers.  DIR = -1 forward, +1 inverse.
// ---------------------------------------------------------------------------
template <class T, int DIR> __device__ __forceinline__ void bfly2(Cx<T>* v) {
    Cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}

template <class T, int DIR> __device__ __forceinline__ void bfly3(Cx<T>* v) {
    const T h = (T)0.86602540378443864676;  // sqrt(3)/2
    Cx<T> t1 = v[1] + v[2], t2 = v[1] - v[2];
    Cx<T> y0 = v[0] + t1;
    Cx<T> mm = v[0] - (T)0.5 * t1;
    Cx<T> u = mul_si<T, DIR>(h * t2);
    v[0] = y0;
    v[1] = mm + u;
    v[2] = mm - u;
}

template <class T, int DIR> __device__ __forceinline__ void bfly4(Cx<T>* v) {
    Cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2], t2 = v[1] + v[3];
    Cx<T> t3 = mul_si<T, DIR>(v[1] - v[3]);
    v[0] = t0 + t2;
    v[2] = t0 - t2;
    v[1] = t1 + t3;
    v[3] = t1 - t3;
}

template <class T, int DIR> __device__ __forceinline__ void bfly5(Cx<T>* v) {
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    Cx<T> t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
    Cx<T> a1 = v[0] + c1 * t1 + c2 * t2;
    Cx<T> a2 = v[0] + c2 * t1 + c1 * t2;
    Cx<T> b1 = mul_si<T, DIR>(s1 * t3 + s2 * t4);
    Cx<T> b2 = mul_si<T, DIR>(s2 * t3 - s1 * t4);
    v[0] = v[0] + t1 + t2;
    v[1] = a1 + b1;
    v[4] = a1 - b1;
    v[2] = a2 + b2;
    v[3] = a2 - b2;
}

template <class T, int DIR> __device__ __forceinline__ void bfly8(Cx<T>* v) {
    Cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    Cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    bfly4<T, DIR>(e);
    bfly4<T, DIR>(o);
    const T r = (T)0.70710678118654752440;
    // w8^k = exp(DIR 2 pi i k / 8)
    Cx<T> w1 = {r, (T)DIR * r}, w3 = {-r, (T)DIR * r};
    Cx<T> o1 = w1 * o[1], o2 = mul_si<T, DIR>(o[2]), o3 = w3 * o[3];
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + o1;
    v[5] = e[1] - o1;
    v[2] = e[2] + o2;
    v[6] = e[2] - o2;
    v[3] = e[3] + o3;
    v[7] = e[3] - o3;
}

// 16 points: the 8-point transforms of the even and odd samples and one
// radix-2 step with the twiddles w16^k = exp(DIR 2 pi i k / 16).
template <class T, int DIR> __device__ __forceinline__ void bfly16(Cx<T>* v) {
    Cx<T> e[8], o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        e[k] = v[2 * k];
        o[k] = v[2 * k + 1];
    }
    bfly8<T, DIR>(e);
    bfly8<T, DIR>(o);
    const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173, r = (T)0.70710678118654752440;
    const Cx<T> w[8] = {{1, 0}, {c1, (T)DIR * s1}, {r, (T)DIR * r}, {s1, (T)DIR * c1},
                        {0, (T)DIR}, {-s1, (T)DIR * c1}, {-r, (T)DIR * r}, {-c1, (T)DIR * s1}};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const Cx<T> t = k == 0 ? o[0] : (k == 4 ? mul_si<T, DIR>(o[4]) : w[k] * o[k]);
        v[k] = e[k] + t;
        v[k + 8] = e[k] - t;
    }
}

template <class T, int DIR, int R> __device__ __forceinline__ void bfly(Cx<T>* v) {
    if constexpr (R == 2) bfly2<T, DIR>(v);
    else if constexpr (R == 3) bfly3<T, DIR>(v);
    else if constexpr (R == 4) bfly4<T, DIR>(v);
    else if constexpr (R == 5) bfly5<T, DIR>(v);
    else if constexpr (R == 16) bfly16<T, DIR>(v);
    else bfly8<T, DIR>(v);
}

// ---------------------------------------------------------------------------
// FFT plan: the length and its radix factorisation (applied in order).
// ---------------------------------------------------------------------------
struct FftPlan {
    int n;
    int np;
    int r[8];
};

// Address of line l in an LDS batch: (l / lg) * ls1 + (l % lg) * ls0.
struct LineAddr {
    int lg, ls0, ls1;
    __device__ __forceinline__ int operator()(int l) const { return (l / lg) * ls1 + (l % lg) * ls0; }
};

// One Stockham radix-R pass over `nl` lines of length n held in LDS, in place:
// every thread first reads and transforms up to MAXB butterflies into
// registers, the block synchronises, then all results are written.  Lines are
// the fastest-varying butterfly index so that neighbouring lanes touch
// neighbouring lines (bank-conflict free for odd line pitches).
// tw[i] = exp(-2 pi i idx / n) (forward table; conjugated for DIR = +1).
template <class T, int DIR, int R, int MAXB>
__device__ __forceinline__ void fft_pass(Cx<T>* buf, int n, int nl, int L, LineAddr la, int es,
                                         const Cx<T>* tw, int tid, int nth) {
    const int nb = n / R;
    const int tot = nb * nl;
    const int tws = n / (L * R);
    Cx<T> v[MAXB][R];
#pragma unroll
    for (int c = 0; c < MAXB; ++c) {
        const int b = tid + c * nth;
        if (b < tot) {
            const int l = b % nl, j = b / nl;
            const int base = la(l);
            const int k = j % L;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                Cx<T> a = buf[base + (j + t * nb) * es];
                if (t > 0 && k > 0) {
                    Cx<T> w = tw[t * k * tws];
                    if (DIR > 0) w.im = -w.im;
                    a = a * w;
                }
                v[c][t] = a;
            }
            bfly<T, DIR, R>(v[c]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < MAXB; ++c) {
        const int b = tid + c * nth;
        if (b < tot) {
            const int l = b % nl, j = b / nl;
            const int base = la(l);
            const int k = j % L;
            const int ob = (j - k) * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) buf[base + (ob + t * L) * es] = v[c][t];
        }
    }
    __syncthreads();
}

// Full FFT of `nl` LDS lines (natural order in, natural order out).  The
// caller must have synchronised after writing the lines.  Requires
// (n / r_min) * nl <= MAXB * nth, checked by the host when it picks nth.
template <class T, int DIR, int MAXB>
__device__ void fft_lines(Cx<T>* buf, const FftPlan& p, int nl, LineAddr la, int es, const Cx<T>* tw,
                          int tid, int nth) {
    int L = 1;
    for (int s = 0; s < p.np; ++s) {
        const int R = p.r[s];
        switch (R) {
            case 2: fft_pass<T, DIR, 2, MAXB>(buf, p.n, nl, L, la, es, tw, tid, nth); break;
            case 3: fft_pass<T, DIR, 3, MAXB>(buf, p.n, nl, L, la, es, tw, tid, nth); break;
            case 4: fft_pass<T, DIR, 4, MAXB>(buf, p.n, nl, L, la, es, tw, tid, nth); break;
            case 5: fft_pass<T, DIR, 5, MAXB>(buf, p.n, nl, L, la, es, tw, tid, nth); break;
            default: fft_pass<T, DIR, 8, MAXB>(buf, p.n, nl, L, la, es, tw, tid, nth); break;
        }
        L *= R;
    }
}

// Complex quotient and product of FP64 scalars held as double2 (re, im).
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------------------
// Wave-level and block-level reductions (64-wide wavefronts).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Value from another lane of the same row of 16 by a DPP row operation
// (CTRL: quad permutation or row mirror).  Every lane of the wave must be
// active.
template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave, the same bits in every lane, without LDS
// traffic (a shuffle of a double is two LDS permutes): DPP steps within rows
// of 16 lanes, each pairing lanes that hold equal partial sums (quad swaps,
// half-row mirror, row mirror), then the four row sums from lanes 0, 16, 32
// and 48 in a fixed order.  Every lane of the wave must be active.
__device__ __forceinline__ double wave_total(double v) {
    v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x141>(v);  // row_half_mirror
    v += dpp_d<0x140>(v);  // row_mirror
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Sums of NV values over the block with one barrier; results valid in
// thread 0 (v is overwritten).  `sh` needs NV * blockDim.x / 64 doubles;
// blockDim.x is a multiple of 64 and every thread takes part.
template <int NV>
__device__ __forceinline__ void block_sum_n(double* v, double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_total(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[w * NV + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = 0;
            for (int k = 0; k < nw; ++k) s += sh[k * NV + i];
            v[i] = s;
        }
}

// Sum of `v` over the block; result valid in thread 0.  `sh` needs
// blockDim.x / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) s += sh[i];
    }
    return s;
}

// ---------------------------------------------------------------------------
// Compile-time FFT: line length, radix plan, number of lines, threads and
// LDS addressing are template constants, so every index is a shift or a
// multiply by a constant and the per-thread butterfly registers are sized
// exactly.  Same Stockham scheme as fft_pass above.
// ---------------------------------------------------------------------------
template <int N> struct RadixPlan;
template <> struct RadixPlan<2> { static constexpr int np = 1; static constexpr int r[1] = {2}; };
template <> struct RadixPlan<4> { static constexpr int np = 1; static constexpr int r[1] = {4}; };
template <> struct RadixPlan<8> { static constexpr int np = 1; static constexpr int r[1] = {8}; };
template <> struct RadixPlan<16> { static constexpr int np = 2; static constexpr int r[2] = {4, 4}; };
template <> struct RadixPlan<32> { static constexpr int np = 2; static constexpr int r[2] = {8, 4}; };
template <> struct RadixPlan<48> { static constexpr int np = 3; static constexpr int r[3] = {3, 4, 4}; };
template <> struct RadixPlan<64> { static constexpr int np = 2; static constexpr int r[2] = {8, 8}; };
template <> struct RadixPlan<96> { static constexpr int np = 3; static constexpr int r[3] = {3, 8, 4}; };
template <> struct RadixPlan<128> { static constexpr int np = 2; static constexpr int r[2] = {16, 8}; };
template <> struct RadixPlan<256> { static constexpr int np = 3; static constexpr int r[3] = {8, 8, 4}; };

// Line l of the LDS batch starts at (l / LG) * LS1 + (l % LG) * LS0; its
// elements are ES apart.  KEEP < N (last step only): outputs KEEP .. N - 1
// of each line are not written (nor, where the compiler can drop them,
// computed); the last step writes output j + t L of its butterfly j, so
// output t of every butterfly is kept iff t L < KEEP.
template <class T, int DIR, int N, int R, int L, int NL, int NTH, int LG, int LS0, int LS1, int ES, int KEEP = N>
__device__ __forceinline__ void ct_pass(Cx<T>* __restrict__ buf, const Cx<T>* __restrict__ tw, int tid) {
    constexpr int NB = N / R, TOT = NB * NL, MB = (TOT + NTH - 1) / NTH, TWS = N / (L * R);
    static_assert(KEEP == N || (L * R == N && KEEP % L == 0 && KEEP < N), "pruned outputs only in the last step");
    Cx<T> v[MB][R];
#pragma unroll
    for (int c = 0; c < MB; ++c) {
        const int b = tid + c * NTH;
        if ((TOT % NTH) == 0 || b < TOT) {
            const int l = b % NL, j = b / NL;
            const int base = (l / LG) * LS1 + (l % LG) * LS0;
            const int k = j % L;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                Cx<T> a = buf[base + (j + t * NB) * ES];
                if (L > 1 && t > 0) {
                    Cx<T> w = tw[t * k * TWS];
                    if (DIR > 0) w.im = -w.im;
                    a = a * w;
                }
                v[c][t] = a;
            }
            bfly<T, DIR, R>(v[c]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < MB; ++c) {
        const int b = tid + c * NTH;
        if ((TOT % NTH) == 0 || b < TOT) {
            const int l = b % NL, j = b / NL;
            const int base = (l / LG) * LS1 + (l % LG) * LS0;
            const int k = j % L;
            const int ob = (j - k) * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t)
                if (t * L < KEEP) buf[base + (ob + t * L) * ES] = v[c][t];
        }
    }
    __syncthreads();
}

template <class T, int DIR, int N, int NL, int NTH, int LG, int LS0, int LS1, int ES, int KEEP, int P, int L>
__device__ __forceinline__ void ct_fft_steps(Cx<T>* __restrict__ buf, const Cx<T>* __restrict__ tw, int tid) {
    if constexpr (P < RadixPlan<N>::np) {
        constexpr int R = RadixPlan<N>::r[P];
        constexpr int K = (P + 1 == RadixPlan<N>::np) ? KEEP : N;
        ct_pass<T, DIR, N, R, L, NL, NTH, LG, LS0, LS1, ES, K>(buf, tw, tid);
        ct_fft_steps<T, DIR, N, NL, NTH, LG, LS0, LS1, ES, KEEP, P + 1, L * R>(buf, tw, tid);
    }
}

template <class T, int DIR, int N, int NL, int NTH, int LG, int LS0, int LS1, int ES>
__device__ __forceinline__ void ct_fft(Cx<T>* __restrict__ buf, const Cx<T>* __restrict__ tw, int tid) {
    ct_fft_steps<T, DIR, N, NL, NTH, LG, LS0, LS1, ES, N, 0, 1>(buf, tw, tid);
}

// As ct_fft, writing only outputs 0 .. KEEP - 1 of each line.
template <class T, int DIR, int N, int NL, int NTH, int LG, int LS0, int LS1, int ES, int KEEP>
__device__ __forceinline__ void ct_fft_keep(Cx<T>* __restrict__ buf, const Cx<T>* __restrict__ tw, int tid) {
    ct_fft_steps<T, DIR, N, NL, NTH, LG, LS0, LS1, ES, KEEP, 0, 1>(buf, tw, tid);
}
