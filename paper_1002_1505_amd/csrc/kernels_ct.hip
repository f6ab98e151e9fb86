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

template <int N> constexpr int plane_threads() { return N >= 128 ? 1024 : 256; }
template <int N> constexpr int zpass_threads() { return N >= 128 ? 512 : 256; }

template <class T, int N>
__global__ void __launch_bounds__(plane_threads<N>()) k_pfwd_ct(const Cx<T>* __restrict__ x, Cx<T>* __restrict__ slab,
                                                                Geo g, Tw<T> tw, int nrhs, const int* __restrict__ active) {
    constexpr int NTH = plane_threads<N>();
    constexpr int PITCH = N + 1;
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* t1 = reinterpret_cast<Cx<T>*>(smem_raw);
    Cx<T>* buf = t1 + N;
    const int nplanes = nrhs * 3 * N;
    const int b = blockIdx.x;
    const int plane = ((b >> 3) >> 2) * 8 + (b & 7);
    const int par = (b >> 3) & 3;
    if (plane >= nplanes) return;
    const int rhs = plane / (3 * N);
    if (active && !active[rhs]) return;
    const int c = (plane / N) % 3, z = plane % N;
    const int px = par & 1, py = par >> 1;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += NTH) t1[i] = tw.f1[i];
    for (int i = tid; i < N * PITCH; i += NTH) buf[i] = Cx<T>{0, 0};
    __syncthreads();
    const Cx<T>* xv = x + ((size_t)rhs * 3 + c) * g.Npad;
    const int j0 = g.plane_start[z], j1 = g.plane_start[z + 1];
    for (int j = j0 + tid; j < j1; j += NTH) {
        const uint32_t s = g.site_xyz[j];
        const int sx = s & 1023, sy = (s >> 10) & 1023;
        Cx<T> v = xv[j];
        if (px) v = v * tw.h1[sx];
        if (py) v = v * tw.h2[sy];
        buf[sy * PITCH + sx] = v;
    }
    __syncthreads();
    ct_fft<T, -1, N, N, NTH, N, PITCH, 0, 1>(buf, t1, tid);   // along x: lines are rows
    ct_fft<T, -1, N, N, NTH, N, 1, 0, PITCH>(buf, t1, tid);   // along y: lines are columns
    Cx<T>* out = slab + ((((size_t)rhs * 3 + c) * N + z) * 4 + par) * (size_t)(N * N);
    for (int i = tid; i < N * N; i += NTH) out[i] = buf[(i / N) * PITCH + (i % N)];
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

template <class T, int N, int MODE>
__global__ void __launch_bounds__(plane_threads<N>()) k_pinv_ct(const Cx<T>* __restrict__ slab, const Cx<T>* __restrict__ x,
                                                                Cx<T>* __restrict__ y, const Cx<T>* __restrict__ bvec,
                                                                const Cx<T>* __restrict__ ainv, Geo g, Tw<T> tw, int nrhs,
                                                                const int* __restrict__ active) {
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
    if (plane >= nplanes) return;
    const int rhs = plane / (3 * N);
    if (active && !active[rhs]) return;
    const int c = (plane / N) % 3, z = plane % N;
    const int qx = q & 1, qy = q >> 1;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += NTH) t1[i] = tw.f1[i];
    const Cx<T>* in = slab + (((size_t)rhs * 3 + c) * N + z) * 4 * (size_t)NN;
    const T sgx = qx ? (T)-1 : (T)1, sgy = qy ? (T)-1 : (T)1;
    for (int e = tid; e < NN; e += NTH) {
        const int kyp = e / N, kxp = e % N;
        const int bx = kxp >> 1, px = kxp & 1, by = kyp >> 1, py = kyp & 1;
        const Cx<T>* blk = in + (size_t)(py * 2 + px) * NN;
        const Cx<T> s00 = blk[by * N + bx], s10 = blk[by * N + bx + HN];
        const Cx<T> s01 = blk[(by + HN) * N + bx], s11 = blk[(by + HN) * N + bx + HN];
        Cx<T> v = s00 + sgx * s10 + sgy * (s01 + sgx * s11);
        if (qx) v = cmulc(tw.h1[kxp], v);
        if (qy) v = cmulc(tw.h2[kyp], v);
        buf[kyp * PITCH + kxp] = v;
    }
    __syncthreads();
    ct_fft<T, +1, N, N, NTH, N, 1, 0, PITCH>(buf, t1, tid);    // along y, every column
    ct_fft<T, +1, N, HN, NTH, HN, PITCH, 0, 1>(buf, t1, tid);  // along x, rows y' < n/2
    const size_t vo = ((size_t)rhs * 3 + c) * g.Npad;
    const Cx<T>* av = ainv + (size_t)rhs * g.ncomp;
    const int j0 = g.plane_start[z], j1 = g.plane_start[z + 1];
    for (int j = j0 + tid; j < j1; j += NTH) {
        const uint32_t s = g.site_xyz[j];
        const int sx = s & 1023, sy = (s >> 10) & 1023;
        if ((sx & 1) != qx || (sy & 1) != qy) continue;
        const Cx<T> v = buf[(sy >> 1) * PITCH + (sx >> 1)] + av[g.site_comp[j]] * x[vo + j];
        if (MODE == MV_AX) y[vo + j] = v;
        else y[vo + j] = bvec[vo + j] - v;
    }
}

template <class T, int N>
constexpr size_t plane_lds() { return (size_t)(N + N * (N + 1)) * sizeof(Cx<T>); }
template <class T, int N, int TX>
constexpr size_t zpass_lds() { return (size_t)(N + 6 * N * TX) * sizeof(Cx<T>); }
constexpr size_t LDS_MAX = 160 * 1024;

template <class T, int N>
hipError_t pass_n(int which, int tx, const Geo& g, const Tw<T>& tw, int nrhs, const Cx<T>* x, Cx<T>* y,
                  const Cx<T>* b, Cx<T>* slab, const Cx<T>* ghat, const Cx<T>* ainv, const int* active, int mode,
                  hipStream_t st) {
    const int nplanes = nrhs * 3 * N;
    const int nblk_plane = (nplanes + 7) / 8 * 8 * 4;
    if (which == 0 || which == 2) {
        if constexpr (plane_lds<T, N>() > LDS_MAX) {
            return hipErrorNotSupported;
        } else {
            if (which == 0) {
                hipLaunchKernelGGL((k_pfwd_ct<T, N>), dim3(nblk_plane), dim3(plane_threads<N>()), (plane_lds<T, N>()), st,
                                   x, slab, g, tw, nrhs, active);
            } else if (mode == MV_AX) {
                hipLaunchKernelGGL((k_pinv_ct<T, N, MV_AX>), dim3(nblk_plane), dim3(plane_threads<N>()),
                                   (plane_lds<T, N>()), st, slab, x, y, b, ainv, g, tw, nrhs, active);
            } else {
                hipLaunchKernelGGL((k_pinv_ct<T, N, MV_RESID>), dim3(nblk_plane), dim3(plane_threads<N>()),
                                   (plane_lds<T, N>()), st, slab, x, y, b, ainv, g, tw, nrhs, active);
            }
            return hipGetLastError();
        }
    }
    const int ntile = 4 * N * N;
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
        e = hipFuncSetAttribute((const void*)k_pfwd_ct<T, N>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_pinv_ct<T, N, MV_AX>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_pinv_ct<T, N, MV_RESID>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    lim);
    }
    if constexpr (zpass_lds<T, N, 8>() <= LDS_MAX && N % 8 == 0)
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_zpass_ct<T, N, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if constexpr (zpass_lds<T, N, 16>() <= LDS_MAX && N % 16 == 0)
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_zpass_ct<T, N, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if constexpr (zpass_lds<T, N, 32>() <= LDS_MAX && N % 32 == 0)
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_zpass_ct<T, N, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    return e;
}

}  // namespace

bool ct_supported(int n1, int n2, int n3) {
    if (n1 != n2 || n2 != n3) return false;
    return n1 == 16 || n1 == 32 || n1 == 48 || n1 == 64 || n1 == 128;
}

template <class T>
hipError_t launch_pass_ct(int which, int tx, const Geo& g, const Tw<T>& tw, int nrhs, const Cx<T>* x, Cx<T>* y,
                          const Cx<T>* b, Cx<T>* slab, const Cx<T>* ghat, const Cx<T>* ainv, const int* active,
                          int mode, hipStream_t st) {
    if (!ct_supported(g.n1, g.n2, g.n3)) return hipErrorNotSupported;
    switch (g.n1) {
        case 16: return pass_n<T, 16>(which, tx, g, tw, nrhs, x, y, b, slab, ghat, ainv, active, mode, st);
        case 32: return pass_n<T, 32>(which, tx, g, tw, nrhs, x, y, b, slab, ghat, ainv, active, mode, st);
        case 48: return pass_n<T, 48>(which, tx, g, tw, nrhs, x, y, b, slab, ghat, ainv, active, mode, st);
        case 64: return pass_n<T, 64>(which, tx, g, tw, nrhs, x, y, b, slab, ghat, ainv, active, mode, st);
        default: return pass_n<T, 128>(which, tx, g, tw, nrhs, x, y, b, slab, ghat, ainv, active, mode, st);
    }
}

// Which passes of a cubic box of side n have a specialised kernel in precision
// T with z tile tx: bit 0 planes, bit 1 z pass.
template <class T>
int ct_available(int n, int tx) {
    auto planes = [](size_t lds) { return lds <= LDS_MAX; };
    int bits = 0;
    if (!ct_supported(n, n, n)) return 0;
    if (planes((size_t)(n + n * (n + 1)) * sizeof(Cx<T>))) bits |= 1;
    if ((tx == 8 || tx == 16 || tx == 32) && n % tx == 0 && (size_t)(n + 6 * n * tx) * sizeof(Cx<T>) <= LDS_MAX)
        bits |= 2;
    return bits;
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

template hipError_t launch_pass_ct<float>(int, int, const Geo&, const Tw<float>&, int, const Cx<float>*, Cx<float>*,
                                          const Cx<float>*, Cx<float>*, const Cx<float>*, const Cx<float>*, const int*,
                                          int, hipStream_t);
template hipError_t launch_pass_ct<double>(int, int, const Geo&, const Tw<double>&, int, const Cx<double>*,
                                           Cx<double>*, const Cx<double>*, Cx<double>*, const Cx<double>*,
                                           const Cx<double>*, const int*, int, hipStream_t);
template int ct_available<float>(int, int);
template int ct_available<double>(int, int);
