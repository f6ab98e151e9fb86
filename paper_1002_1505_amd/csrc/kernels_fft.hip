// FFT-accelerated DDA matrix-vector product on gfx950.
//
// The off-diagonal part of A (a convolution with the dipole interaction
// tensor, Goodman, Draine & Flatau 1991) is applied on the doubled grid
// M_i = 2 n_i.  Each doubled axis is split by frequency parity: with
// k = 2k' + p, the M-point DFT of data that is zero beyond n equals an
// n-point DFT of the data pre-multiplied by exp(-2 pi i p x / M).  Every
// transform is then an unpadded n-point FFT and the spectrum is stored as
// 2 x 2 x 2 parity blocks of n1 x n2 x n3.
//
// Three passes per matvec (one launch each, all right-hand sides):
//   1. xy forward: per (rhs, component, z, parity px py): scatter the sites of
//      plane z into LDS with the pre-twiddles, 2D FFT, write the parity block.
//   2. z pass: per tile of (kx, ky) columns: both z parities, z FFT, 3x3
//      multiply by the symmetric tensor spectrum, inverse z FFT, recombine.
//   3. xy inverse: per (rhs, component, z): inverse 2D FFT of the four parity
//      blocks, post-twiddle and sum, then gather at the occupied sites and add
//      the diagonal 1/alpha P (or form b - A x).
// A fallback keeps the plane in global memory (scatter, line FFTs, gather)
// when an n1 x n2 plane does not fit the 160 KB LDS.
#include "dda_internal.h"

#define HIP_TRY(x)                             \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return e_;       \
    } while (0)

namespace {

constexpr int MAXB = 4;  // butterflies per thread per pass
constexpr int EPT = 16;  // plane elements per thread in the inverse pass

// ---------------------------------------------------------------------------
// Pass 1: scatter + 2D forward FFT of one parity block of one plane.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(1024) k_plane_fwd(const Cx<T>* __restrict__ x, Cx<T>* __restrict__ slab, Geo g,
                                                    Tw<T> tw, FftPlan p1, FftPlan p2, int nrhs,
                                                    const int* __restrict__ active) {
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* sm = reinterpret_cast<Cx<T>*>(smem_raw);
    const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
    const int nplanes = nrhs * 3 * n3;
    // The four parity blocks of one plane get block ids with equal id % 8 so
    // that they run on the same XCD and share its L2 for the input plane.
    const int b = blockIdx.x;
    const int plane = ((b >> 3) >> 2) * 8 + (b & 7);
    const int par = (b >> 3) & 3;
    if (plane >= nplanes) return;
    const int rhs = plane / (3 * n3);
    if (active && !active[rhs]) return;
    const int c = (plane / n3) % 3, z = plane % n3;
    const int px = par & 1, py = par >> 1;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int pitch = n1 + 1;
    Cx<T>* t1 = sm;
    Cx<T>* t2 = t1 + n1;
    Cx<T>* buf = t2 + n2;
    for (int i = tid; i < n1; i += nth) t1[i] = tw.f1[i];
    for (int i = tid; i < n2; i += nth) t2[i] = tw.f2[i];
    for (int i = tid; i < n2 * pitch; i += nth) buf[i] = Cx<T>{0, 0};
    __syncthreads();
    const Cx<T>* xv = x + ((size_t)rhs * 3 + c) * g.Npad;
    const int j0 = g.plane_start[z], j1 = g.plane_start[z + 1];
    for (int j = j0 + tid; j < j1; j += nth) {
        const uint32_t s = g.site_xyz[j];
        const int sx = s & 1023, sy = (s >> 10) & 1023;
        Cx<T> v = xv[j];
        if (px) v = v * tw.h1[sx];
        if (py) v = v * tw.h2[sy];
        buf[sy * pitch + sx] = v;
    }
    __syncthreads();
    fft_lines<T, -1, MAXB>(buf, p1, n2, LineAddr{n2, pitch, 0}, 1, t1, tid, nth);
    fft_lines<T, -1, MAXB>(buf, p2, n1, LineAddr{n1, 1, 0}, pitch, t2, tid, nth);
    Cx<T>* out = slab + ((((size_t)rhs * 3 + c) * n3 + z) * 4 + par) * (size_t)(n1 * n2);
    for (int i = tid; i < n1 * n2; i += nth) {
        const int yy = i / n1, xx = i - yy * n1;
        out[i] = buf[yy * pitch + xx];
    }
}

// ---------------------------------------------------------------------------
// Pass 2: z FFT (both parities), tensor multiply, inverse z FFT.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ int fold_index(int k, int n, int& sgn) {
    // k in [0, 2n): folded frequency f = min(k, 2n - k), stored at
    // (f & 1) * (n/2 + 1) + (f >> 1); sgn = -1 beyond the midpoint.
    int f = k;
    sgn = 1;
    if (k > n) {
        f = 2 * n - k;
        sgn = -1;
    }
    return (f & 1) * (n / 2 + 1) + (f >> 1);
}

template <class T>
__global__ void __launch_bounds__(1024) k_zpass(Cx<T>* __restrict__ slab, const Cx<T>* __restrict__ gh, Geo g,
                                                Tw<T> tw, FftPlan p3, int nrhs, int TX,
                                                const int* __restrict__ active) {
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* sm = reinterpret_cast<Cx<T>*>(smem_raw);
    const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
    const int ncol = 4 * n1 * n2;
    const int ntile = ncol / TX;
    const int rhs = blockIdx.x / ntile, tile = blockIdx.x - rhs * ntile;
    if (rhs >= nrhs) return;
    if (active && !active[rhs]) return;
    const int q0 = tile * TX;
    const int par = q0 / (n1 * n2), rem = q0 - par * (n1 * n2);
    const int px = par & 1, py = par >> 1;
    const int kyp = rem / n1, kx0 = rem - kyp * n1;
    const int tid = threadIdx.x, nth = blockDim.x;
    Cx<T>* t3 = sm;
    Cx<T>* W = t3 + n3;
    const int E = 3 * n3 * TX;
    for (int i = tid; i < n3; i += nth) t3[i] = tw.f3[i];
    Cx<T>* base = slab + (size_t)rhs * 3 * n3 * ncol + q0;
    for (int e = tid; e < E; e += nth) {
        const int col = e % TX, cz = e / TX;  // cz = c * n3 + z
        const int z = cz % n3;
        const Cx<T> v = base[(size_t)cz * ncol + col];
        W[e] = v;
        W[E + e] = v * tw.h3[z];
    }
    __syncthreads();
    fft_lines<T, -1, MAXB>(W, p3, 6 * TX, LineAddr{TX, 1, n3 * TX}, TX, t3, tid, nth);
    // Tensor multiply.  Spectrum octant layout: [comp][kz][ky][kx], each
    // folded axis stored as parity * (n/2+1) + f/2.
    const int Dx = 2 * (n1 / 2 + 1), Dy = 2 * (n2 / 2 + 1), Dz = 2 * (n3 / 2 + 1);
    const size_t cs = (size_t)Dx * Dy * Dz;
    int sy;
    const int kyi = fold_index<T>(2 * kyp + py, n2, sy);
    for (int i = tid; i < 2 * n3 * TX; i += nth) {
        const int col = i % TX, zz = i / TX;
        const int kzp = zz % n3, pz = zz / n3;
        Cx<T>* w = W + pz * E;
        int sx, sz;
        const int kxi = fold_index<T>(2 * (kx0 + col) + px, n1, sx);
        const int kzi = fold_index<T>(2 * kzp + pz, n3, sz);
        const size_t gi = ((size_t)kzi * Dy + kyi) * Dx + kxi;
        const Cx<T> gxx = gh[gi], gxy = (T)(sx * sy) * gh[cs + gi], gxz = (T)(sx * sz) * gh[2 * cs + gi];
        const Cx<T> gyy = gh[3 * cs + gi], gyz = (T)(sy * sz) * gh[4 * cs + gi], gzz = gh[5 * cs + gi];
        const int o0 = kzp * TX + col, o1 = (n3 + kzp) * TX + col, o2 = (2 * n3 + kzp) * TX + col;
        const Cx<T> a0 = w[o0], a1 = w[o1], a2 = w[o2];
        w[o0] = gxx * a0 + gxy * a1 + gxz * a2;
        w[o1] = gxy * a0 + gyy * a1 + gyz * a2;
        w[o2] = gxz * a0 + gyz * a1 + gzz * a2;
    }
    __syncthreads();
    fft_lines<T, +1, MAXB>(W, p3, 6 * TX, LineAddr{TX, 1, n3 * TX}, TX, t3, tid, nth);
    for (int e = tid; e < E; e += nth) {
        const int col = e % TX, cz = e / TX;
        const int z = cz % n3;
        base[(size_t)cz * ncol + col] = W[e] + cmulc(tw.h3[z], W[E + e]);
    }
}

// ---------------------------------------------------------------------------
// Pass 3: inverse 2D FFT of the four parity blocks, recombination, gather and
// diagonal term.
// ---------------------------------------------------------------------------
template <class T, int MODE>
__global__ void __launch_bounds__(1024) k_plane_inv(const Cx<T>* __restrict__ slab, const Cx<T>* __restrict__ x,
                                                    Cx<T>* __restrict__ y, const Cx<T>* __restrict__ bvec,
                                                    const Cx<T>* __restrict__ ainv, Geo g, Tw<T> tw, FftPlan p1,
                                                    FftPlan p2, int nrhs, const int* __restrict__ active) {
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* sm = reinterpret_cast<Cx<T>*>(smem_raw);
    const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
    const int plane = blockIdx.x;
    const int rhs = plane / (3 * n3);
    if (rhs >= nrhs) return;
    if (active && !active[rhs]) return;
    const int c = (plane / n3) % 3, z = plane % n3;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int pitch = n1 + 1;
    const int np = n1 * n2;
    Cx<T>* t1 = sm;
    Cx<T>* t2 = t1 + n1;
    Cx<T>* buf = t2 + n2;
    for (int i = tid; i < n1; i += nth) t1[i] = tw.f1[i];
    for (int i = tid; i < n2; i += nth) t2[i] = tw.f2[i];
    Cx<T> acc[EPT];
    const Cx<T>* in = slab + (((size_t)rhs * 3 + c) * n3 + z) * 4 * (size_t)np;
    for (int par = 0; par < 4; ++par) {
        const int px = par & 1, py = par >> 1;
        for (int i = tid; i < np; i += nth) {
            const int yy = i / n1, xx = i - yy * n1;
            buf[yy * pitch + xx] = in[(size_t)par * np + i];
        }
        __syncthreads();
        fft_lines<T, +1, MAXB>(buf, p2, n1, LineAddr{n1, 1, 0}, pitch, t2, tid, nth);
        fft_lines<T, +1, MAXB>(buf, p1, n2, LineAddr{n2, pitch, 0}, 1, t1, tid, nth);
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = tid + k * nth;
            if (e < np) {
                const int yy = e / n1, xx = e - yy * n1;
                Cx<T> v = buf[yy * pitch + xx];
                if (px) v = cmulc(tw.h1[xx], v);
                if (py) v = cmulc(tw.h2[yy], v);
                acc[k] = (par == 0) ? v : acc[k] + v;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = tid + k * nth;
        if (e < np) {
            const int yy = e / n1, xx = e - yy * n1;
            buf[yy * pitch + xx] = acc[k];
        }
    }
    __syncthreads();
    const size_t vo = ((size_t)rhs * 3 + c) * g.Npad;
    const Cx<T>* av = ainv + (size_t)rhs * g.ncomp;
    const int j0 = g.plane_start[z], j1 = g.plane_start[z + 1];
    for (int j = j0 + tid; j < j1; j += nth) {
        const uint32_t s = g.site_xyz[j];
        const int sx = s & 1023, sy = (s >> 10) & 1023;
        const Cx<T> v = buf[sy * pitch + sx] + av[g.site_comp[j]] * x[vo + j];
        if (MODE == MV_AX) y[vo + j] = v;
        else y[vo + j] = bvec[vo + j] - v;
    }
}

// ---------------------------------------------------------------------------
// Fallback for planes larger than LDS: scatter, line FFTs, gather.
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(Cx<T>* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = Cx<T>{0, 0};
}

template <class T>
__global__ void k_scatter_par(const Cx<T>* __restrict__ x, Cx<T>* __restrict__ slab, Geo g, Tw<T> tw, int nrhs,
                              const int* __restrict__ active) {
    const int rhs = blockIdx.y / 3, c = blockIdx.y % 3;
    if (active && !active[rhs]) return;
    const int np = g.n1 * g.n2;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < g.N; j += gridDim.x * blockDim.x) {
        const uint32_t s = g.site_xyz[j];
        const int sx = s & 1023, sy = (s >> 10) & 1023, sz = s >> 20;
        const Cx<T> v = x[((size_t)rhs * 3 + c) * g.Npad + j];
        Cx<T>* o = slab + ((((size_t)rhs * 3 + c) * g.n3 + sz) * 4) * (size_t)np + sy * g.n1 + sx;
        const Cx<T> vx = v * tw.h1[sx], vy = v * tw.h2[sy];
        o[0] = v;
        o[np] = vx;
        o[2 * (size_t)np] = vy;
        o[3 * (size_t)np] = vx * tw.h2[sy];
    }
}

template <class T, int MODE>
__global__ void k_gather_par(const Cx<T>* __restrict__ slab, const Cx<T>* __restrict__ x, Cx<T>* __restrict__ y,
                             const Cx<T>* __restrict__ bvec, const Cx<T>* __restrict__ ainv, Geo g, Tw<T> tw,
                             int nrhs, const int* __restrict__ active) {
    const int rhs = blockIdx.y / 3, c = blockIdx.y % 3;
    if (active && !active[rhs]) return;
    const int np = g.n1 * g.n2;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < g.N; j += gridDim.x * blockDim.x) {
        const uint32_t s = g.site_xyz[j];
        const int sx = s & 1023, sy = (s >> 10) & 1023, sz = s >> 20;
        const Cx<T>* o = slab + ((((size_t)rhs * 3 + c) * g.n3 + sz) * 4) * (size_t)np + sy * g.n1 + sx;
        const Cx<T> hx = tw.h1[sx], hy = tw.h2[sy];
        Cx<T> v = o[0] + cmulc(hx, o[np]) + cmulc(hy, o[2 * (size_t)np]) + cmulc(hx * hy, o[3 * (size_t)np]);
        const size_t vi = ((size_t)rhs * 3 + c) * g.Npad + j;
        v = v + ainv[(size_t)rhs * g.ncomp + g.site_comp[j]] * x[vi];
        if (MODE == MV_AX) y[vi] = v;
        else y[vi] = bvec[vi] - v;
    }
}

// FFT of lines through global memory: line l = (o, i) with o = l / inner,
// i = l % inner; element e at o * os + e * es + i * is.  TL lines per block.
template <class T, int DIR>
__global__ void __launch_bounds__(1024) k_lines(Cx<T>* __restrict__ data, long long nlines, long long inner,
                                                long long os, long long es, long long is, FftPlan p,
                                                const Cx<T>* __restrict__ twg, int TL,
                                                const int* __restrict__ active, long long lines_per_rhs) {
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* sm = reinterpret_cast<Cx<T>*>(smem_raw);
    const int n = p.n;
    const int tid = threadIdx.x, nth = blockDim.x;
    const long long l0 = (long long)blockIdx.x * TL;
    if (active) {
        const long long r0 = l0 / lines_per_rhs, r1 = (l0 + TL - 1) / lines_per_rhs;
        if (r0 == r1 && !active[r0]) return;
    }
    Cx<T>* t = sm;
    Cx<T>* buf = t + n;
    const int pitch = n + 1;
    for (int i = tid; i < n; i += nth) t[i] = twg[i];
    const bool colmode = (is == 1);
    for (int idx = tid; idx < TL * n; idx += nth) {
        int li, e;
        if (colmode) {
            li = idx % TL;
            e = idx / TL;
        } else {
            e = idx % n;
            li = idx / n;
        }
        const long long l = l0 + li;
        if (l < nlines) {
            const long long o = l / inner, ii = l - o * inner;
            buf[li * pitch + e] = data[o * os + e * es + ii * is];
        }
    }
    __syncthreads();
    fft_lines<T, DIR, MAXB>(buf, p, TL, LineAddr{TL, pitch, 0}, 1, t, tid, nth);
    for (int idx = tid; idx < TL * n; idx += nth) {
        int li, e;
        if (colmode) {
            li = idx % TL;
            e = idx / TL;
        } else {
            e = idx % n;
            li = idx / n;
        }
        const long long l = l0 + li;
        if (l < nlines) {
            const long long o = l / inner, ii = l - o * inner;
            data[o * os + e * es + ii * is] = buf[li * pitch + e];
        }
    }
}

// ---------------------------------------------------------------------------
// Green's tensor spectrum (FP64).
// ---------------------------------------------------------------------------
// Off-diagonal interaction block A(d) for lattice separation d != 0:
//   exp(ikr)/r [k^2 (nn - I) + (ikr - 1)/r^2 (3 nn - I)],
// six unique components xx, xy, xz, yy, yz, zz.
__device__ void interaction(double dx, double dy, double dz, double k, Cx<double>* a) {
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double r = sqrt(r2);
    const double nx = dx / r, ny = dy / r, nz = dz / r;
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const Cx<double> ph = {cs / r, sn / r};
    const Cx<double> c2 = {-1.0 / r2, k / r};  // (ikr - 1)/r^2
    const double k2 = k * k;
    const double nn[6] = {nx * nx, nx * ny, nx * nz, ny * ny, ny * nz, nz * nz};
    const double id[6] = {1, 0, 0, 1, 0, 1};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const Cx<double> t = {k2 * (nn[q] - id[q]) + c2.re * (3 * nn[q] - id[q]), c2.im * (3 * nn[q] - id[q])};
        a[q] = ph * t;
    }
}

// work[q][par8][jz][jy][jx]: the pre-combined parity inputs whose n-point 3D
// FFTs give the M-point spectrum at k = 2 k' + p (for each axis).
__global__ void k_green_par(Geo g, double kd, Tw<double> tw, Cx<double>* __restrict__ work) {
    const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
    const long long nn = (long long)n1 * n2 * n3;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nn) return;
    const int jx = id % n1, jy = (id / n1) % n2, jz = id / ((long long)n1 * n2);
    Cx<double> lag[8][6];
    for (int s = 0; s < 8; ++s) {
        const int ix = jx + (s & 1) * n1, iy = jy + ((s >> 1) & 1) * n2, iz = jz + (s >> 2) * n3;
        // lag on the circulant grid; the unused lag +-n and the zero lag are 0
        const bool zero = (ix == n1) || (iy == n2) || (iz == n3) || (ix == 0 && iy == 0 && iz == 0);
        if (zero) {
            for (int q = 0; q < 6; ++q) lag[s][q] = Cx<double>{0, 0};
        } else {
            const double dx = ix < n1 ? ix : ix - 2 * n1;
            const double dy = iy < n2 ? iy : iy - 2 * n2;
            const double dz = iz < n3 ? iz : iz - 2 * n3;
            interaction(dx, dy, dz, kd, lag[s]);
        }
    }
    for (int p = 0; p < 8; ++p) {
        Cx<double> w = {1, 0};
        if (p & 1) w = w * tw.h1[jx];
        if (p & 2) w = w * tw.h2[jy];
        if (p & 4) w = w * tw.h3[jz];
        for (int q = 0; q < 6; ++q) {
            Cx<double> acc = {0, 0};
            for (int s = 0; s < 8; ++s) {
                const int sg = __popc(p & s) & 1;
                acc = sg ? acc - lag[s][q] : acc + lag[s][q];
            }
            work[((size_t)q * 8 + p) * nn + id] = w * acc;
        }
    }
}

__global__ void k_green_oct(Geo g, const Cx<double>* __restrict__ work, Cx<double>* __restrict__ g64,
                            Cx<float>* __restrict__ g32, double scale) {
    const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
    const long long nn = (long long)n1 * n2 * n3;
    const int Dx = 2 * (n1 / 2 + 1), Dy = 2 * (n2 / 2 + 1), Dz = 2 * (n3 / 2 + 1);
    const long long tot = 6LL * Dx * Dy * Dz;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= tot) return;
    const int xi = id % Dx, yi = (id / Dx) % Dy, zi = (id / ((long long)Dx * Dy)) % Dz;
    const int q = id / ((long long)Dx * Dy * Dz);
    // invert the folded-parity index: slot = parity * (n/2+1) + f/2
    const int hx = n1 / 2 + 1, hy = n2 / 2 + 1, hz = n3 / 2 + 1;
    const int fx = 2 * (xi % hx) + xi / hx, fy = 2 * (yi % hy) + yi / hy, fz = 2 * (zi % hz) + zi / hz;
    Cx<double> v = {0, 0};
    if (fx <= n1 && fy <= n2 && fz <= n3) {
        const int p = (fx & 1) | ((fy & 1) << 1) | ((fz & 1) << 2);
        const long long j = (long long)(fz >> 1) * n1 * n2 + (long long)(fy >> 1) * n1 + (fx >> 1);
        v = scale * work[((size_t)q * 8 + p) * nn + j];
    }
    g64[id] = v;
    if (g32) g32[id] = Cx<float>{(float)v.re, (float)v.im};
}

template <class T>
int lines_nth(const FftPlan& p, int TL) {
    int rmin = 8;
    for (int s = 0; s < p.np; ++s) rmin = p.r[s] < rmin ? p.r[s] : rmin;
    const int bf = (p.n / rmin) * TL;
    int nth = (bf + MAXB - 1) / MAXB;
    nth = ((nth + 63) / 64) * 64;
    if (nth < 64) nth = 64;
    return nth;
}

template <class T, int DIR>
hipError_t run_lines(Cx<T>* data, long long nlines, long long inner, long long os, long long es, long long is,
                     const FftPlan& p, const Cx<T>* tw, int TL, const int* active, long long lines_per_rhs,
                     hipStream_t st) {
    const int nth = lines_nth<T>(p, TL);
    if (nth > 1024) return hipErrorInvalidConfiguration;
    const size_t sh = (size_t)(p.n + TL * (p.n + 1)) * sizeof(Cx<T>);
    const unsigned nb = (unsigned)((nlines + TL - 1) / TL);
    hipLaunchKernelGGL((k_lines<T, DIR>), dim3(nb), dim3(nth), sh, st, data, nlines, inner, os, es, is, p, tw, TL,
                       active, lines_per_rhs);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <class T>
static size_t plane_smem(const Geo& g) {
    return (size_t)(g.n1 + g.n2 + g.n2 * (g.n1 + 1)) * sizeof(Cx<T>);
}
template <class T>
static size_t zpass_smem(const Geo& g, int tx) {
    return (size_t)(g.n3 + 2 * 3 * g.n3 * tx) * sizeof(Cx<T>);
}
static int rmin_of(const FftPlan& p) {
    int r = 8;
    for (int s = 0; s < p.np; ++s) r = p.r[s] < r ? p.r[s] : r;
    return r;
}

template <class T>
bool matvec_shape_ok(const Geo& g, const FftPlan* plans, const MvShape& sh) {
    const size_t lds_max = 160 * 1024;
    if (sh.zrb < 0 || sh.zrb > 4) return false;
    if (sh.zrb >= 2 && !(sh.ct & 2)) return false;
    if (sh.ct) {
        if (g.n1 != g.n2 || g.n2 != g.n3) return false;
        const int av = ct_available<T>(g.n1, sh.tx);
        if ((sh.ct & av) != sh.ct) return false;
        if ((sh.ct & 2) && !ct_zpass_fits<T>(g.n1, sh.tx, sh.zrb)) return false;
        if ((sh.ct & 4) && !(sh.ct & 1)) return false;
        if ((sh.ct & 8) && ((sh.ct & 3) != 3 || (sh.zrb != 3 && sh.zrb != 4))) return false;
        if ((sh.ct & 3) == 3) return true;
    }
    if (sh.tx <= 0 || (g.n1 % sh.tx) != 0) return false;
    if (zpass_smem<T>(g, sh.tx) > lds_max) return false;
    const int bz = (g.n3 / rmin_of(plans[2])) * 6 * sh.tx;
    if (bz > MAXB * sh.nth_z || sh.nth_z > 1024 || (sh.nth_z % 64)) return false;
    if (sh.fused) {
        if (plane_smem<T>(g) > lds_max) return false;
        const int np = g.n1 * g.n2;
        if (np > EPT * sh.nth_plane || sh.nth_plane > 1024 || (sh.nth_plane % 64)) return false;
        const int bx = (g.n1 / rmin_of(plans[0])) * g.n2, by = (g.n2 / rmin_of(plans[1])) * g.n1;
        if (bx > MAXB * sh.nth_plane || by > MAXB * sh.nth_plane) return false;
    } else {
        if (lines_nth<T>(plans[0], sh.lines_tl) > 1024 || lines_nth<T>(plans[1], sh.lines_tl) > 1024) return false;
    }
    return true;
}

template <class T>
hipError_t launch_pass(int which, const Geo& g, const Tw<T>& tw, const FftPlan* plans, const MvShape& sh, int nrhs,
                       const Cx<T>* x, Cx<T>* y, const Cx<T>* b, Cx<T>* slab, const Cx<T>* ghat, const Cx<T>* ainv,
                       const int* active, int mode, hipStream_t st, MvDot dot, MvUpd upd) {
    const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
    const long long np = (long long)n1 * n2;
    if ((which == 1 && (sh.ct & 2)) || (which != 1 && (sh.ct & 1)))
        return launch_pass_ct<T>(which, sh.tx, sh.zrb, sh.ct, g, tw, nrhs, x, y, b, slab, ghat, ainv, active, mode,
                                 which == 2 ? dot.dot : 0, (const Cx<T>*)dot.w, dot.partials, upd, st);
    if (which == 0) {
        if (sh.fused) {
            const int nplanes = nrhs * 3 * n3;
            const int nplanes8 = (nplanes + 7) / 8 * 8;
            hipLaunchKernelGGL((k_plane_fwd<T>), dim3(nplanes8 * 4), dim3(sh.nth_plane), plane_smem<T>(g), st, x,
                               slab, g, tw, plans[0], plans[1], nrhs, active);
            return hipGetLastError();
        }
        const size_t tot = (size_t)nrhs * 3 * n3 * 4 * np;
        hipLaunchKernelGGL((k_fill<T>), dim3(2048), dim3(256), 0, st, slab, tot);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL((k_scatter_par<T>), dim3((g.N + 255) / 256, nrhs * 3), dim3(256), 0, st, x, slab, g, tw,
                           nrhs, active);
        HIP_TRY(hipGetLastError());
        const long long blocks = (long long)nrhs * 3 * n3 * 4;
        // x lines: rows of each parity block
        HIP_TRY((run_lines<T, -1>(slab, blocks * n2, 1, n1, 1, 0, plans[0], tw.f1, sh.lines_tl, active,
                                  3LL * n3 * 4 * n2, st)));
        // y lines: columns of each parity block
        return run_lines<T, -1>(slab, blocks * n1, n1, np, n1, 1, plans[1], tw.f2, sh.lines_tl, active,
                                3LL * n3 * 4 * n1, st);
    }
    if (which == 1) {
        const int ntile = 4 * n1 * n2 / sh.tx;
        hipLaunchKernelGGL((k_zpass<T>), dim3(nrhs * ntile), dim3(sh.nth_z), zpass_smem<T>(g, sh.tx), st, slab, ghat,
                           g, tw, plans[2], nrhs, sh.tx, active);
        return hipGetLastError();
    }
    if (sh.fused) {
        if (mode == MV_AX)
            hipLaunchKernelGGL((k_plane_inv<T, MV_AX>), dim3(nrhs * 3 * n3), dim3(sh.nth_plane), plane_smem<T>(g), st,
                               slab, x, y, b, ainv, g, tw, plans[0], plans[1], nrhs, active);
        else
            hipLaunchKernelGGL((k_plane_inv<T, MV_RESID>), dim3(nrhs * 3 * n3), dim3(sh.nth_plane), plane_smem<T>(g),
                               st, slab, x, y, b, ainv, g, tw, plans[0], plans[1], nrhs, active);
        return hipGetLastError();
    }
    const long long blocks = (long long)nrhs * 3 * n3 * 4;
    HIP_TRY((run_lines<T, +1>(slab, blocks * n1, n1, np, n1, 1, plans[1], tw.f2, sh.lines_tl, active,
                              3LL * n3 * 4 * n1, st)));
    HIP_TRY((run_lines<T, +1>(slab, blocks * n2, 1, n1, 1, 0, plans[0], tw.f1, sh.lines_tl, active,
                              3LL * n3 * 4 * n2, st)));
    if (mode == MV_AX)
        hipLaunchKernelGGL((k_gather_par<T, MV_AX>), dim3((g.N + 255) / 256, nrhs * 3), dim3(256), 0, st, slab, x, y, b,
                           ainv, g, tw, nrhs, active);
    else
        hipLaunchKernelGGL((k_gather_par<T, MV_RESID>), dim3((g.N + 255) / 256, nrhs * 3), dim3(256), 0, st, slab, x,
                           y, b, ainv, g, tw, nrhs, active);
    return hipGetLastError();
}

template <class T>
hipError_t launch_matvec(const Geo& g, const Tw<T>& tw, const FftPlan* plans, const MvShape& sh, int nrhs,
                         const Cx<T>* x, Cx<T>* y, const Cx<T>* b, Cx<T>* slab, const Cx<T>* ghat, const Cx<T>* ainv,
                         const int* active, int mode, hipStream_t st, MvDot dot, MvUpd upd) {
    if ((dot.dot || upd.mode) && !(sh.ct & 1)) return hipErrorNotSupported;
    // A large batch of a small box runs its three passes chunk by chunk, the
    // chunk's slab (at most MV_CHUNK_BYTES) staying in the 256 MB last-level
    // cache from the pass that writes it to the pass that reads it.  Every
    // per-rhs array keeps its stride (vectors 3 Npad, 1/alpha ncomp, fused
    // partials 4 x 12 n complex, states and flags one), so a chunk is the
    // same launch on offset pointers, and each rhs's arithmetic is unchanged.
    const size_t slab_rhs = (size_t)12 * g.n1 * g.n2 * g.n3 * sizeof(Cx<T>);
    const int chunk = (int)std::min<size_t>((size_t)nrhs, MV_CHUNK_BYTES / slab_rhs);
    if (chunk >= 4 && chunk < nrhs) {
        const size_t ve = (size_t)3 * g.Npad, ps = (size_t)4 * 12 * g.n1 * 2;
        for (int r0 = 0; r0 < nrhs; r0 += chunk) {
            const int nr = std::min(chunk, nrhs - r0);
            MvDot d = dot;
            if (d.w) d.w = reinterpret_cast<const Cx<T>*>(d.w) + r0 * ve;
            if (d.partials) d.partials += r0 * ps;
            MvUpd u = upd;
            if (u.r) u.r = reinterpret_cast<const Cx<T>*>(u.r) + r0 * ve;
            if (u.v) u.v = reinterpret_cast<const Cx<T>*>(u.v) + r0 * ve;
            if (u.pout) u.pout = reinterpret_cast<Cx<T>*>(u.pout) + r0 * ve;
            if (u.st) u.st += r0;
            if (u.part) u.part += r0 * ps;
            for (int w = 0; w < 3; ++w)
                HIP_TRY(launch_pass<T>(w, g, tw, plans, sh, nr, x + r0 * ve, y + r0 * ve, b ? b + r0 * ve : nullptr,
                                       slab, ghat, ainv + (size_t)r0 * g.ncomp, active ? active + r0 : nullptr, mode,
                                       st, d, u));
        }
        return hipSuccess;
    }
    for (int w = 0; w < 3; ++w)
        HIP_TRY(launch_pass<T>(w, g, tw, plans, sh, nrhs, x, y, b, slab, ghat, ainv, active, mode, st, dot, upd));
    return hipSuccess;
}

template <class T>
__global__ void k_green_interleave(const Cx<T>* __restrict__ gh, Cx<T>* __restrict__ gz, size_t cs, int hx) {
    const int H1 = hx + 1, Dx = 2 * H1;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cs; i += (size_t)gridDim.x * blockDim.x) {
        size_t o = i;
        if (hx) {  // x columns in the order of the class-grouped slab's groups
            const int xi = (int)(i % Dx), half = xi / H1;
            o = i - xi + half * H1 + spec_xpos(xi % H1, half, hx);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) gz[o * 6 + q] = gh[q * cs + i];
    }
}

template <class T>
hipError_t launch_green_interleave(const Cx<T>* gh, Cx<T>* gz, size_t cs, int hx, hipStream_t st) {
    hipLaunchKernelGGL((k_green_interleave<T>), dim3(1024), dim3(256), 0, st, gh, gz, cs, hx);
    return hipGetLastError();
}
template hipError_t launch_green_interleave<float>(const Cx<float>*, Cx<float>*, size_t, int, hipStream_t);
template hipError_t launch_green_interleave<double>(const Cx<double>*, Cx<double>*, size_t, int, hipStream_t);

hipError_t launch_green(const Geo& g, const Tw<double>& tw, const FftPlan* plans, double kd, Cx<double>* work,
                        Cx<double>* g64, Cx<float>* g32, hipStream_t st) {
    const long long nn = (long long)g.n1 * g.n2 * g.n3;
    hipLaunchKernelGGL(k_green_par, dim3((unsigned)((nn + 127) / 128)), dim3(128), 0, st, g, kd, tw, work);
    HIP_TRY(hipGetLastError());
    const long long nb = 48;  // 6 components x 8 parity blocks
    const long long np = (long long)g.n1 * g.n2;
    // x: rows; y: columns within planes; z: columns across planes
    HIP_TRY((run_lines<double, -1>(work, nb * g.n3 * g.n2, 1, g.n1, 1, 0, plans[0], tw.f1, 16, nullptr, 1LL << 62, st)));
    HIP_TRY((run_lines<double, -1>(work, nb * g.n3 * g.n1, g.n1, np, g.n1, 1, plans[1], tw.f2, 16, nullptr, 1LL << 62,
                                   st)));
    HIP_TRY((run_lines<double, -1>(work, nb * np, np, nn, np, 1, plans[2], tw.f3, 16, nullptr, 1LL << 62, st)));
    const long long tot = (long long)ghat_octant_elems(g.n1, g.n2, g.n3);
    const double scale = 1.0 / (8.0 * (double)nn);
    hipLaunchKernelGGL(k_green_oct, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, g, work, g64, g32, scale);
    return hipGetLastError();
}

template hipError_t launch_matvec<float>(const Geo&, const Tw<float>&, const FftPlan*, const MvShape&, int,
                                         const Cx<float>*, Cx<float>*, const Cx<float>*, Cx<float>*, const Cx<float>*,
                                         const Cx<float>*, const int*, int, hipStream_t, MvDot, MvUpd);
template hipError_t launch_matvec<double>(const Geo&, const Tw<double>&, const FftPlan*, const MvShape&, int,
                                          const Cx<double>*, Cx<double>*, const Cx<double>*, Cx<double>*,
                                          const Cx<double>*, const Cx<double>*, const int*, int, hipStream_t, MvDot, MvUpd);
template hipError_t launch_pass<float>(int, const Geo&, const Tw<float>&, const FftPlan*, const MvShape&, int,
                                       const Cx<float>*, Cx<float>*, const Cx<float>*, Cx<float>*, const Cx<float>*,
                                       const Cx<float>*, const int*, int, hipStream_t, MvDot, MvUpd);
template hipError_t launch_pass<double>(int, const Geo&, const Tw<double>&, const FftPlan*, const MvShape&, int,
                                        const Cx<double>*, Cx<double>*, const Cx<double>*, Cx<double>*,
                                        const Cx<double>*, const Cx<double>*, const int*, int, hipStream_t, MvDot, MvUpd);
template bool matvec_shape_ok<float>(const Geo&, const FftPlan*, const MvShape&);
template bool matvec_shape_ok<double>(const Geo&, const FftPlan*, const MvShape&);

// Allow the LDS-heavy kernels to use the 160 KB of LDS of a gfx950 CU.
hipError_t configure_fft_kernels() {
    const int lim = 160 * 1024;
    HIP_TRY(set_lds_limit((const void*)k_plane_fwd<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    HIP_TRY(set_lds_limit((const void*)k_plane_fwd<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    HIP_TRY(set_lds_limit((const void*)k_zpass<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    HIP_TRY(set_lds_limit((const void*)k_zpass<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    HIP_TRY(set_lds_limit((const void*)k_plane_inv<float, MV_AX>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    HIP_TRY(set_lds_limit((const void*)k_plane_inv<float, MV_RESID>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    HIP_TRY(set_lds_limit((const void*)k_plane_inv<double, MV_AX>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    HIP_TRY(set_lds_limit((const void*)k_plane_inv<double, MV_RESID>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    HIP_TRY(set_lds_limit((const void*)k_lines<float, -1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    HIP_TRY(set_lds_limit((const void*)k_lines<float, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    HIP_TRY(set_lds_limit((const void*)k_lines<double, -1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    HIP_TRY(set_lds_limit((const void*)k_lines<double, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    return hipSuccess;
}
