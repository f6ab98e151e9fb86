// Host runtime and C ABI of the DDA solver (see include/dda.h).
//
// A context owns the targets (site lists, twiddles, tensor spectra, tuned
// launch shapes) and the workspace of the last solve.  A solve groups its
// right-hand sides by target; every kernel launch covers all right-hand sides
// of a group, and one BiCGstab iteration of all groups is captured in a HIP
// graph that is replayed several iterations at a time between convergence
// polls.  FP32_REFINE runs the Krylov iteration on FP32 vectors and the FP32
// matvec, recomputes the residual b - A x with the FP64 matvec, and refines x
// in FP64 until the FP64 residual meets the tolerance.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/dda.h"
#include "dda_internal.h"

using cd = std::complex<double>;

hipError_t nn_record_one(dda_nn* nn, const NnSiteView& tv, const dda_wave& w, const double* ainv,
                         const Cx<double>* x64, const Cx<float>* esh, const Cx<float>* rf, float rscale,
                         hipStream_t st);
hipError_t nn_guess_group(dda_nn* nn, const NnSiteView& t, const dda_wave* waves, const double* ainv, int nr,
                          const Cx<float>* esh, const Cx<float>* rf, const double* rn2, Cx<double>* x64,
                          hipStream_t st);

namespace {

constexpr double PI = 3.14159265358979323846;
// Lattice-dispersion-relation coefficients (Draine & Goodman 1993).
constexpr double LDR_B1 = -1.8915316, LDR_B2 = 0.1648469, LDR_B3 = -1.7700004;

struct DevMem {
    void* p = nullptr;
    size_t n = 0;
    unsigned gen = 0;  // allocations so far (a new allocation may reuse the old address)
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t ensure(size_t bytes) {
        if (bytes <= n && p) return hipSuccess;
        release();
        if (!bytes) return hipSuccess;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        n = bytes;
        ++gen;
        return hipSuccess;
    }
    template <class U>
    U* as() const { return reinterpret_cast<U*>(p); }
};

// Pinned host memory, grown on demand: asynchronous copies from it return at
// once (pageable sources are staged by the runtime and block the caller).
// Contents must stay untouched until the copies that read them complete.
struct PinMem {
    void* p = nullptr;
    size_t n = 0;
    PinMem() = default;
    PinMem(const PinMem&) = delete;
    PinMem& operator=(const PinMem&) = delete;
    ~PinMem() { release(); }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t ensure(size_t bytes) {
        if (bytes <= n && p) return hipSuccess;
        release();
        hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        n = bytes;
        return hipSuccess;
    }
    template <class U> U* as() const { return static_cast<U*>(p); }
};

struct Target {
    long long uid = 0;
    int n[3] = {0, 0, 0};
    int N = 0, Npad = 0, ncomp = 0;
    std::vector<cd> m;
    // anisotropic compositions: principal refractive indices and the
    // Dielectric Frame angles (Theta_DF, Phi_DF, beta_DF); aniso[c] = 0 for
    // isotropic compositions
    std::vector<char> aniso;
    std::vector<std::array<cd, 3>> m3;
    std::vector<std::array<double, 3>> dfang;
    bool any_aniso = false;
    double kd = 0;
    int alpha_kind = DDA_ALPHA_LDR;
    double origin[3] = {0, 0, 0};
    double aeff = 0;
    FftPlan plans[3];
    DevMem d_xyz, d_comp, d_pstart, d_cstart, d_perm, tw64, tw32, gh64, gh32;
    DevMem gz64, gz32;  // n = 64, 128: spectrum with components interleaved (two-factor z passes)
    DevMem gz64g, gz32g;  // the same with x columns in the class-grouped slab's group order
    DevMem zt16, zt32, zt16g;  // n = 64: z-pass tile order per XCD
    DevMem zt8, zt8g;          // n = 128: the same for 8-column tiles (row and grouped layouts)
    bool have64 = false, have32 = false;
    MvShape sh32{}, sh64{};
    Geo geo() const {
        Geo g;
        g.n1 = n[0];
        g.n2 = n[1];
        g.n3 = n[2];
        g.N = N;
        g.Npad = Npad;
        g.ncomp = ncomp;
        g.plane_start = d_pstart.as<int>();
        g.class_start = d_cstart.as<int>();
        g.perm = d_perm.as<int>();
        g.ztiles16 = zt16.as<int>();
        g.ztiles32 = zt32.as<int>();
        g.ztiles16g = zt16g.as<int>();
        g.ztiles8 = zt8.as<int>();
        g.ztiles8g = zt8g.as<int>();
        g.site_xyz = d_xyz.as<uint32_t>();
        g.site_comp = d_comp.as<uint8_t>();
        return g;
    }
    template <class T>
    Tw<T> tw() const {
        const DevMem& d = std::is_same<T, double>::value ? tw64 : tw32;
        const Cx<T>* b = d.as<Cx<T>>();
        Tw<T> t;
        t.f1 = b;
        t.f2 = t.f1 + n[0];
        t.f3 = t.f2 + n[1];
        t.h1 = t.f3 + n[2];
        t.h2 = t.h1 + n[0];
        t.h3 = t.h2 + n[1];
        return t;
    }
    template <class T>
    const MvShape& shape() const { return std::is_same<T, double>::value ? sh64 : sh32; }
    template <class T>
    const Cx<T>* ghat() const {
        return std::is_same<T, double>::value ? gh64.as<Cx<T>>() : gh32.as<Cx<T>>();
    }
    // spectrum layout the launch shape's z pass reads
    template <class T>
    const Cx<T>* ghat_for(const MvShape& sh) const {
        if (sh.ct & 8) return std::is_same<T, double>::value ? gz64g.as<Cx<T>>() : gz32g.as<Cx<T>>();
        if ((sh.ct & 2) && sh.zrb >= 2)
            return std::is_same<T, double>::value ? gz64.as<Cx<T>>() : gz32.as<Cx<T>>();
        return ghat<T>();
    }
};

// Workspace of the right-hand sides of one solve that share a target.
struct Group {
    int tgt = -1, nr = 0, kprec = 0;
    std::vector<int> idx;  // call-level rhs index of each member
    DevMem waves, ainv64, ainv32, b64, x64, r64;
    DevMem kv[8];  // inner Krylov vectors x r rhat p v s t p' (kprec precision)
    DevMem slab32, slab64;
    DevMem state, active, partials, scale, tolrel2, maxit, norms, mask;
    // tensor 1/alpha of anisotropic compositions per (slot, composition), 6
    // complex (xx, xy, xz, yy, yz, zz), zero for isotropic ones
    DevMem aten64, aten32;
    std::vector<cd> haten;
    std::vector<Cx<float>> haten32;
    // per-iteration recursive residuals of the inner solve (DDA_TRACE), [nr][tcap]
    DevMem trace;
    int tcap = 0;
    // previous solve of the same slots: waves and 1/alpha; the local field
    // (1/alpha) P0 of the least-squares guess, its residual field E - A P0
    // (FP32) and the rms of that residual per slot, inputs of the learned guess
    DevMem wprev, ainvprev, esh, rf, rfn2;  // rfn2: ||E - A P0||^2 per slot (FP32 field, FP64 sum)
    std::vector<float> hrscale;
    bool has_r = false;
    // ring of the last `hdepth` solutions of every slot with their waves and
    // 1/alpha (filled by solves with history > 0), and the scratch of the
    // least-squares guess over it
    DevMem hx[HIST_MAX], hwv[HIST_MAX], hainvv[HIST_MAX];
    int hdepth = 0, hn = 0, hhead = 0;
    DevMem pv32, pw32, pcoef, gpart;
    // host staging buffers of asynchronous uploads (must outlive the copies)
    std::vector<WaveDev> hw;
    std::vector<cd> hainv;  // [nr][ncomp]
    std::vector<Cx<float>> hainv32;
    std::vector<int> hmask;
    // pinned staging of the refinement loop: per-slot scale and squared
    // tolerance (double), iteration budget and mask (int); inner-solve states
    PinMem hup, hst;
    double* up_scale() const { return hup.as<double>(); }
    double* up_tol2() const { return hup.as<double>() + nr; }
    int* up_maxit() const { return reinterpret_cast<int*>(hup.as<double>() + 2 * nr); }
    int* up_mask() const { return up_maxit() + nr; }
    size_t up_bytes() const { return (size_t)nr * (2 * sizeof(double) + 2 * sizeof(int)); }
};

}  // namespace

struct dda_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    std::vector<std::unique_ptr<Target>> tg;
    std::vector<std::unique_ptr<Group>> groups;
    int last_nrhs = 0;
    std::vector<int> rhs_group, rhs_slot;
    bool have_solution = false;
    // graph cache
    // captured inner iterations, one per set of groups that still iterate
    // (a group whose rhs have all stopped is left out of the replays)
    std::map<std::vector<char>, hipGraphExec_t> gexec;
    long long gkey_gen = -1;
    int gkey_prec = 0, gkey_k = 0;
    void drop_graphs() {
        for (auto& kv : gexec) (void)hipGraphExecDestroy(kv.second);
        gexec.clear();
    }
    long long ws_gen = 0;
    dda_nn* nn = nullptr;  // learned-guess model (not owned)
    std::vector<dda_wave> last_waves;
    double ms_guess = 0;
    // test hook of the solve options: forced restart period of the inner BiCGstab
    int force_restart = 0;
    // inner Krylov method (DDA_SOLVER_*) of the solve in progress
    int solver = 0;
    int gkey_solver = -1;
    // DDA_TRACE: file receiving the per-iteration residuals of every solve
    std::string trace_path;
    long long ncalls = 0;
    // timing
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // convergence polls of the inner solve: active flags of every group
    // copied into pinned host memory, two slots, one event per slot
    int* poll_host = nullptr;
    size_t poll_cap = 0;
    hipEvent_t evpoll[2] = {nullptr, nullptr};
    double ms_mv32 = 0, ms_mv64 = 0, ms_total = 0;
    // device scratch of the post-solve calls (cross sections, amplitudes,
    // moments), kept between calls: no allocation or free per call
    DevMem scr[8];
};

namespace {

dda_status fail(dda_ctx* c, dda_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HCHK(ctx, x)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (x);                                                                         \
        if (e_ != hipSuccess)                                                                        \
            return fail(ctx, e_ == hipErrorOutOfMemory ? DDA_ERR_OOM : DDA_ERR_HIP, "%s failed: %s (%s:%d)", \
                        #x, hipGetErrorString(e_), __FILE__, __LINE__);                              \
    } while (0)

#define SCHK(x)                              \
    do {                                     \
        dda_status s_ = (x);                 \
        if (s_ < 0) return s_;               \
    } while (0)

bool factor_plan(int n, FftPlan& p) {
    p.n = n;
    p.np = 0;
    int a = 0, b = 0, c = 0, m = n;
    while (m % 2 == 0) m /= 2, ++a;
    while (m % 3 == 0) m /= 3, ++b;
    while (m % 5 == 0) m /= 5, ++c;
    if (m != 1 || n < 2) return false;
    for (int i = 0; i < c; ++i) p.r[p.np++] = 5;
    for (int i = 0; i < b; ++i) p.r[p.np++] = 3;
    while (a >= 3 && a != 4) p.r[p.np++] = 8, a -= 3;
    if (a == 4) p.r[p.np++] = 4, p.r[p.np++] = 4, a = 0;
    if (a == 2) p.r[p.np++] = 4, a = 0;
    if (a == 1) p.r[p.np++] = 2, a = 0;
    return p.np <= 8;
}

int rmin(const FftPlan& p) {
    int r = 8;
    for (int s = 0; s < p.np; ++s) r = std::min(r, p.r[s]);
    return r;
}
int round64(int x) { return std::max(64, (x + 63) / 64 * 64); }

template <class T>
MvShape default_shape(const Target& t, int tx_pref) {
    const Geo g = t.geo();
    MvShape s{};
    s.lines_tl = 16;
    s.nth_lines = 256;
    // z pass
    int tx = tx_pref;
    while (tx > 1 && (g.n1 % tx != 0)) tx /= 2;
    for (;; tx /= 2) {
        s.tx = tx;
        const int bz = (g.n3 / rmin(t.plans[2])) * 6 * tx;
        s.nth_z = std::max(256, round64((bz + 3) / 4));
        if ((s.nth_z <= 1024 && matvec_shape_ok<T>(g, t.plans, MvShape{0, 64, s.nth_z, tx, 16, 256, 0, 0})) || tx == 1) break;
    }
    // planes
    const int np = g.n1 * g.n2;
    const int bx = (g.n1 / rmin(t.plans[0])) * g.n2, by = (g.n2 / rmin(t.plans[1])) * g.n1;
    int nth = std::max({(np + 15) / 16, (bx + 3) / 4, (by + 3) / 4});
    s.nth_plane = std::max(256, round64(nth));
    s.fused = 1;
    s.ct = 0;
    s.zrb = 0;
    if (!matvec_shape_ok<T>(g, t.plans, s)) s.fused = 0;
    if (ct_supported(g.n1, g.n2, g.n3)) {
        // specialised kernels; z tile 16 columns (8 from n = 128 on, where
        // the generic specialised z pass is faster with narrower tiles)
        // unless only another fits
        MvShape c = s;
        const int txo[3] = {g.n1 >= 128 ? 8 : 16, g.n1 >= 128 ? 16 : 32, g.n1 >= 128 ? 32 : 8};
        for (int txc : txo) {
            c.tx = txc;
            c.ct = ct_available<T>(g.n1, txc);
            if ((c.ct & 2) && matvec_shape_ok<T>(g, t.plans, c)) break;
        }
        if (!(c.ct & 2)) {
            c.tx = s.tx;
            c.ct = ct_available<T>(g.n1, s.tx) & 1;
        }
        // a generic z pass needs its own thread count for the chosen tile
        c.zrb = (c.ct & 2) ? 1 : 0;
        if (c.ct && matvec_shape_ok<T>(g, t.plans, c)) s = c;
        // n = 128, FP32: the two-factor 16 x 8 z pass with one frequency
        // parity per block half, on the class-grouped slab (one load per
        // frequency in the inverse plane pass)
        if (std::is_same<T, float>::value && g.n1 == 128) {
            MvShape c5 = s;
            c5.tx = 8;
            c5.ct = (ct_available<T>(g.n1, 8) & 11);
            c5.zrb = 4;
            if ((c5.ct & 3) == 3 && matvec_shape_ok<T>(g, t.plans, c5)) s = c5;
        }
        // n = 64: the two-factor z pass; in FP32 the variant with one
        // frequency parity per block half (16-column tiles, more waves per
        // SIMD), in FP64 one parity after the other (32-column tiles)
        const int zv[2][2] = {{3, 16}, {2, 32}};
        for (int v = std::is_same<T, double>::value ? 1 : 0; v < 2; ++v) {
            MvShape c3 = s;
            c3.tx = zv[v][1];
            // two-factor inverse plane pass: faster in FP64, on par in FP32;
            // with variant 3 the z pass pre-combines the inverse pass's
            // quadrants (class-grouped slab)
            c3.ct = (ct_available<T>(g.n1, c3.tx) | (s.ct & 1)) & (std::is_same<T, double>::value ? 7 : 11);
            c3.zrb = zv[v][0];
            if (matvec_shape_ok<T>(g, t.plans, c3)) {
                s = c3;
                break;
            }
        }
    }
    return s;
}

// Tile order of the two-factor z pass (cubic box of side n, tiles of tx
// columns): tiles whose columns fold onto the same tensor-spectrum rows form
// a group; groups go whole to the least-loaded XCD, giving [8][tiles / 8].
// In the row layout a tile covers one (parity, ky) row and groups are ky
// with its mirror; in the class-grouped layout (grouped) a tile covers rows
// ky and ky + n, and groups are the pairs {ky, n - ky}.
std::vector<int> zpass_tile_order(int n, int tx, bool grouped) {
    const int ntile = 4 * n * n / tx;
    auto fidx = [n](int k) {
        const int f = k <= n ? k : 2 * n - k;
        return (f & 1) * (n / 2 + 1) + (f >> 1);
    };
    std::vector<std::vector<int>> groups;
    std::map<int, int> gid;  // (parity, smallest folded row) -> group
    for (int tile = 0; tile < ntile; ++tile) {
        const int q0 = tile * tx, par = q0 / (n * n), rem = q0 % (n * n), py = par >> 1;
        int key;
        if (grouped) {
            const int ky = 2 * ((rem >> 2) / (n / 2)) + py;
            key = std::min(fidx(ky), fidx(ky + n));
        } else {
            key = fidx(2 * (rem / n) + py);
        }
        key += par * (n + 2);
        auto it = gid.find(key);
        if (it == gid.end()) {
            it = gid.emplace(key, (int)groups.size()).first;
            groups.emplace_back();
        }
        groups[it->second].push_back(tile);
    }
    std::stable_sort(groups.begin(), groups.end(), [](const std::vector<int>& a, const std::vector<int>& b) {
        return a.size() > b.size();
    });
    std::vector<std::vector<int>> lists(8);
    for (auto& g : groups) {
        int x = 0;
        for (int i = 1; i < 8; ++i)
            if (lists[i].size() < lists[x].size()) x = i;
        lists[x].insert(lists[x].end(), g.begin(), g.end());
    }
    std::vector<int> out;
    for (auto& l : lists) {
        if ((int)l.size() != ntile / 8) return {};  // unbalanced: not used
        out.insert(out.end(), l.begin(), l.end());
    }
    return out;
}

dda_status build_target(dda_ctx* c, Target& t, const int32_t dims[3], const uint8_t* occ, int32_t ncomp,
                        const double* m, double kd, int32_t alpha_kind, const double* origin) {
    if (!dims || !occ || !m || ncomp < 1 || ncomp > 255)
        return fail(c, DDA_ERR_INVALID_ARG, "set_target: null pointer or ncomp out of [1,255]");
    for (int i = 0; i < 3; ++i) {
        if (dims[i] < 2 || dims[i] > 1023) return fail(c, DDA_ERR_UNSUPPORTED_DIMS, "dims[%d]=%d outside [2,1023]", i, dims[i]);
        if (!factor_plan(dims[i], t.plans[i]))
            return fail(c, DDA_ERR_UNSUPPORTED_DIMS, "dims[%d]=%d does not factor into 2, 3 and 5", i, dims[i]);
    }
    if (!(kd > 0) || !std::isfinite(kd)) return fail(c, DDA_ERR_INVALID_ARG, "kd must be positive");
    if (alpha_kind < DDA_ALPHA_CM || alpha_kind > DDA_ALPHA_LDR) return fail(c, DDA_ERR_INVALID_ARG, "bad alpha_kind");
    const int n1 = dims[0], n2 = dims[1], n3 = dims[2];
    // stored order: plane z, then parity class q = 2 (y % 2) + (x % 2), then
    // scan order; perm maps each stored site to its (z, y, x) scan position
    std::vector<uint32_t> xyz;
    std::vector<uint8_t> comp;
    std::vector<int> ps(n3 + 1, 0), cs(4 * n3 + 1, 0), perm;
    double cx = 0, cy = 0, cz = 0;
    int scan = 0;
    std::vector<uint32_t> cls_xyz[4];
    std::vector<uint8_t> cls_comp[4];
    std::vector<int> cls_scan[4];
    for (int z = 0; z < n3; ++z) {
        ps[z] = (int)xyz.size();
        for (int q = 0; q < 4; ++q) {
            cls_xyz[q].clear();
            cls_comp[q].clear();
            cls_scan[q].clear();
        }
        for (int y = 0; y < n2; ++y)
            for (int x = 0; x < n1; ++x) {
                const uint8_t o = occ[(size_t)x + (size_t)n1 * (y + (size_t)n2 * z)];
                if (!o) continue;
                if (o > ncomp) return fail(c, DDA_ERR_INVALID_ARG, "occupancy value %d exceeds ncomp=%d", o, ncomp);
                const int q = 2 * (y & 1) + (x & 1);
                cls_xyz[q].push_back((uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20));
                cls_comp[q].push_back((uint8_t)(o - 1));
                cls_scan[q].push_back(scan++);
                cx += x;
                cy += y;
                cz += z;
            }
        for (int q = 0; q < 4; ++q) {
            cs[4 * z + q] = (int)xyz.size();
            xyz.insert(xyz.end(), cls_xyz[q].begin(), cls_xyz[q].end());
            comp.insert(comp.end(), cls_comp[q].begin(), cls_comp[q].end());
            perm.insert(perm.end(), cls_scan[q].begin(), cls_scan[q].end());
        }
    }
    ps[n3] = (int)xyz.size();
    cs[4 * n3] = (int)xyz.size();
    if (xyz.empty()) return fail(c, DDA_ERR_INVALID_ARG, "target has no occupied site");
    t.n[0] = n1;
    t.n[1] = n2;
    t.n[2] = n3;
    t.N = (int)xyz.size();
    t.Npad = (t.N + 255) / 256 * 256;
    t.ncomp = ncomp;
    t.m.assign(ncomp, cd(0, 0));
    for (int i = 0; i < ncomp; ++i) t.m[i] = cd(m[2 * i], m[2 * i + 1]);
    t.aniso.assign(ncomp, 0);
    t.m3.assign(ncomp, std::array<cd, 3>{});
    t.dfang.assign(ncomp, std::array<double, 3>{});
    t.any_aniso = false;
    t.kd = kd;
    t.alpha_kind = alpha_kind;
    if (origin) {
        for (int i = 0; i < 3; ++i) t.origin[i] = origin[i];
    } else {
        t.origin[0] = cx / t.N;
        t.origin[1] = cy / t.N;
        t.origin[2] = cz / t.N;
    }
    t.aeff = std::cbrt(3.0 * t.N / (4.0 * PI));
    static long long next_uid = 1;
    t.uid = next_uid++;
    HCHK(c, t.d_xyz.ensure(xyz.size() * 4));
    HCHK(c, t.d_comp.ensure(comp.size()));
    HCHK(c, t.d_pstart.ensure(ps.size() * 4));
    HCHK(c, t.d_cstart.ensure(cs.size() * 4));
    HCHK(c, t.d_perm.ensure(perm.size() * 4));
    HCHK(c, hipMemcpy(t.d_xyz.p, xyz.data(), xyz.size() * 4, hipMemcpyHostToDevice));
    HCHK(c, hipMemcpy(t.d_comp.p, comp.data(), comp.size(), hipMemcpyHostToDevice));
    HCHK(c, hipMemcpy(t.d_pstart.p, ps.data(), ps.size() * 4, hipMemcpyHostToDevice));
    HCHK(c, hipMemcpy(t.d_cstart.p, cs.data(), cs.size() * 4, hipMemcpyHostToDevice));
    HCHK(c, hipMemcpy(t.d_perm.p, perm.data(), perm.size() * 4, hipMemcpyHostToDevice));
    t.zt16.release();
    t.zt32.release();
    t.zt16g.release();
    t.zt8.release();
    t.zt8g.release();
    if (n1 == 128 && n2 == 128 && n3 == 128) {
        for (int v = 0; v < 2; ++v) {
            const std::vector<int> order = zpass_tile_order(128, 8, v == 1);
            if (order.empty()) return fail(c, DDA_ERR_UNSUPPORTED_DIMS, "z-pass tile order unbalanced");
            DevMem& d = v ? t.zt8g : t.zt8;
            HCHK(c, d.ensure(order.size() * 4));
            HCHK(c, hipMemcpy(d.p, order.data(), order.size() * 4, hipMemcpyHostToDevice));
        }
    }
    if (n1 == 64 && n2 == 64 && n3 == 64) {
        for (int v = 0; v < 3; ++v) {
            const int tx = v == 1 ? 32 : 16;
            const std::vector<int> order = zpass_tile_order(64, tx, v == 2);
            if (order.empty()) return fail(c, DDA_ERR_UNSUPPORTED_DIMS, "z-pass tile order unbalanced");
            DevMem& d = v == 0 ? t.zt16 : (v == 1 ? t.zt32 : t.zt16g);
            HCHK(c, d.ensure(order.size() * 4));
            HCHK(c, hipMemcpy(d.p, order.data(), order.size() * 4, hipMemcpyHostToDevice));
        }
    }
    // twiddles: f_i (n_i) then h_i (n_i)
    std::vector<Cx<double>> tw;
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < t.n[i]; ++k) {
            const long double a = -2.0L * 3.14159265358979323846264338327950288L * k / t.n[i];
            tw.push_back(Cx<double>{(double)cosl(a), (double)sinl(a)});
        }
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < t.n[i]; ++k) {
            const long double a = -2.0L * 3.14159265358979323846264338327950288L * k / (2 * t.n[i]);
            tw.push_back(Cx<double>{(double)cosl(a), (double)sinl(a)});
        }
    std::vector<Cx<float>> tw32(tw.size());
    for (size_t i = 0; i < tw.size(); ++i) tw32[i] = Cx<float>{(float)tw[i].re, (float)tw[i].im};
    HCHK(c, t.tw64.ensure(tw.size() * sizeof(Cx<double>)));
    HCHK(c, t.tw32.ensure(tw32.size() * sizeof(Cx<float>)));
    HCHK(c, hipMemcpy(t.tw64.p, tw.data(), tw.size() * sizeof(Cx<double>), hipMemcpyHostToDevice));
    HCHK(c, hipMemcpy(t.tw32.p, tw32.data(), tw32.size() * sizeof(Cx<float>), hipMemcpyHostToDevice));
    t.have32 = t.have64 = false;
    t.sh32 = default_shape<float>(t, 16);
    t.sh64 = default_shape<double>(t, 16);
    if (!matvec_shape_ok<float>(t.geo(), t.plans, t.sh32) || !matvec_shape_ok<double>(t.geo(), t.plans, t.sh64))
        return fail(c, DDA_ERR_UNSUPPORTED_DIMS, "no launch shape fits box %dx%dx%d", n1, n2, n3);
    double mkd = 0;
    for (auto& mm : t.m) mkd = std::max(mkd, std::abs(mm) * kd);
    if (mkd >= 1.0) {
        fail(c, DDA_WARN_MKD_GE_1, "|m| k d = %.4f >= 1: outside the validity range of the DDA", mkd);
        return DDA_WARN_MKD_GE_1;
    }
    return DDA_OK;
}

// 1/alpha for composition m at k d = kd (d = 1).
cd inverse_alpha(cd mm, double kd, int kind, const double* khat, const double* e) {
    const cd eps = mm * mm;
    const cd acm = (3.0 / (4.0 * PI)) * (eps - 1.0) / (eps + 2.0);
    cd inv = 1.0 / acm;
    const cd rr = cd(0, -(2.0 / 3.0) * kd * kd * kd);
    if (kind == DDA_ALPHA_CM) return inv;
    if (kind == DDA_ALPHA_CM_RR) return inv + rr;
    double S = 0;
    for (int j = 0; j < 3; ++j) S += khat[j] * khat[j] * (e[2 * j] * e[2 * j] + e[2 * j + 1] * e[2 * j + 1]);
    return inv + (LDR_B1 + eps * LDR_B2 + eps * LDR_B3 * S) * (kd * kd) + rr;
}

// Target-frame tensor 1/alpha of an anisotropic composition: the principal
// axes e_1, e_2, e_3 of its Dielectric Frame (the guide's expansion in the
// Target Frame for angles Theta_DF, Phi_DF, beta_DF), 1/alpha_j from the
// prescription with eps_j = m_j^2 (for LDR with the wave's S, taken in the
// target frame), and 1/alpha = sum_j (1/alpha_j) e_j e_j^T.  out: 6 entries
// (xx, xy, xz, yy, yz, zz).
void aniso_inverse_alpha(const std::array<cd, 3>& m3, const std::array<double, 3>& ang, double kd, int kind,
                         const double* khat, const double* e, cd* out) {
    const double ct = std::cos(ang[0]), st = std::sin(ang[0]), cp = std::cos(ang[1]), sp = std::sin(ang[1]);
    const double cb = std::cos(ang[2]), sb = std::sin(ang[2]);
    const double ax[3][3] = {{ct, st * cp, st * sp},
                             {-st * cb, ct * cb * cp - sb * sp, ct * cb * sp + sb * cp},
                             {st * sb, -(ct * sb * cp + cb * sp), -(ct * sb * sp - cb * cp)}};
    cd inv[3];
    for (int j = 0; j < 3; ++j) inv[j] = inverse_alpha(m3[j], kd, kind, khat, e);
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int q = 0; q < 6; ++q) {
        cd v = 0;
        for (int j = 0; j < 3; ++j) v += inv[j] * (ax[j][ia[q]] * ax[j][ib[q]]);
        out[q] = v;
    }
}

// Tensor and scalar 1/alpha tables of a group for its waves: anisotropic
// compositions get a zero scalar entry (the matvec passes then add nothing)
// and their tensor; isotropic ones a zero tensor.
void aniso_tables(const Target& t, Group& g, const dda_wave* waves_of_slot) {
    g.haten.assign((size_t)g.nr * t.ncomp * 6, cd(0, 0));
    g.haten32.assign(g.haten.size(), Cx<float>{0, 0});
    for (int s = 0; s < g.nr; ++s) {
        const dda_wave& w = waves_of_slot[s];
        for (int q = 0; q < t.ncomp; ++q) {
            if (!t.aniso[q]) continue;
            cd* o = &g.haten[((size_t)s * t.ncomp + q) * 6];
            aniso_inverse_alpha(t.m3[q], t.dfang[q], t.kd, t.alpha_kind, w.khat, w.e0, o);
            for (int k = 0; k < 6; ++k)
                g.haten32[((size_t)s * t.ncomp + q) * 6 + k] = Cx<float>{(float)o[k].real(), (float)o[k].imag()};
            g.hainv[(size_t)s * t.ncomp + q] = 0;
            g.hainv32[(size_t)s * t.ncomp + q] = Cx<float>{0, 0};
        }
    }
}

dda_status check_ctx(dda_ctx* c) {
    if (!c) return DDA_ERR_INVALID_ARG;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return fail(c, DDA_ERR_HIP, "hipSetDevice: %s", hipGetErrorString(e));
    return DDA_OK;
}

NnSiteView site_view(const Target& t) {
    NnSiteView v;
    v.uid = t.uid;
    v.n1 = t.n[0];
    v.n2 = t.n[1];
    v.n3 = t.n[2];
    v.N = t.N;
    v.Npad = t.Npad;
    v.ncomp = t.ncomp;
    v.site_xyz = t.d_xyz.as<uint32_t>();
    v.site_comp = t.d_comp.as<uint8_t>();
    for (int i = 0; i < 3; ++i) v.origin[i] = t.origin[i];
    v.kd = t.kd;
    v.m = reinterpret_cast<const double*>(t.m.data());
    return v;
}

dda_status ensure_green(dda_ctx* c, Target& t, uint32_t prec) {
    const bool need64 = (prec & DDA_FP64) && !t.have64;
    const bool need32 = (prec & DDA_FP32) && !t.have32;
    if (!need64 && !need32) return DDA_OK;
    const size_t oct = ghat_octant_elems(t.n[0], t.n[1], t.n[2]);
    HCHK(c, t.gh64.ensure(oct * sizeof(Cx<double>)));
    if (prec & DDA_FP32 || t.have32) HCHK(c, t.gh32.ensure(oct * sizeof(Cx<float>)));
    DevMem work;
    HCHK(c, work.ensure((size_t)48 * t.n[0] * t.n[1] * t.n[2] * sizeof(Cx<double>)));
    HCHK(c, launch_green(t.geo(), t.tw<double>(), t.plans, t.kd, work.as<Cx<double>>(), t.gh64.as<Cx<double>>(),
                         t.gh32.p ? t.gh32.as<Cx<float>>() : nullptr, c->stream));
    const bool cube = t.n[0] == t.n[1] && t.n[1] == t.n[2];
    if (cube && (t.n[0] == 64 || t.n[0] == 128)) {
        // spectrum with the 6 components of a frequency adjacent (two-factor
        // z passes), also in the class-grouped column order (group half
        // width n/2); at n = 128 only FP32 has a two-factor z pass
        const size_t cs = oct / 6;
        const int hg = t.n[0] / 2;
        for (int hx : {0, hg}) {
            DevMem& d64 = hx ? t.gz64g : t.gz64;
            if (t.n[0] == 64) {
                HCHK(c, d64.ensure(oct * sizeof(Cx<double>)));
                HCHK(c, launch_green_interleave<double>(t.gh64.as<Cx<double>>(), d64.as<Cx<double>>(), cs, hx,
                                                        c->stream));
            }
            if (t.gh32.p) {
                DevMem& d32 = hx ? t.gz32g : t.gz32;
                HCHK(c, d32.ensure(oct * sizeof(Cx<float>)));
                HCHK(c, launch_green_interleave<float>(t.gh32.as<Cx<float>>(), d32.as<Cx<float>>(), cs, hx, c->stream));
            }
        }
    }
    HCHK(c, hipStreamSynchronize(c->stream));
    t.have64 = true;
    if (t.gh32.p) t.have32 = true;
    return DDA_OK;
}

template <class T>
hipError_t matvec_group(const Target& t, Group& g, int nr, const Cx<T>* x, Cx<T>* y, const Cx<T>* b, const int* active,
                        int mode, hipStream_t st, MvDot dot = MvDot{0, nullptr, nullptr},
                        MvUpd upd = MvUpd{0, nullptr, nullptr, nullptr, nullptr, nullptr}) {
    Cx<T>* slab = std::is_same<T, double>::value ? g.slab64.as<Cx<T>>() : g.slab32.as<Cx<T>>();
    const Cx<T>* ainv = std::is_same<T, double>::value ? g.ainv64.as<Cx<T>>() : g.ainv32.as<Cx<T>>();
    // the passes' fused inner products and updates would miss the tensor part
    // of an anisotropic diagonal, which is added after them
    if (t.any_aniso && (dot.dot || upd.mode)) return hipErrorNotSupported;
    hipError_t e = launch_matvec<T>(t.geo(), t.tw<T>(), t.plans, t.shape<T>(), nr, x, y, b, slab,
                                    t.ghat_for<T>(t.shape<T>()), ainv, active, mode, st, dot, upd);
    if (e != hipSuccess || !t.any_aniso) return e;
    const Cx<T>* aten = std::is_same<T, double>::value ? g.aten64.as<Cx<T>>() : g.aten32.as<Cx<T>>();
    return launch_aniso_diag<T>(t.geo(), nr, x, y, aten, mode == MV_RESID ? -1 : 1, st);
}

size_t slab_elems(const Target& t, int nr) { return (size_t)nr * 3 * 4 * t.n[0] * t.n[1] * t.n[2]; }
size_t vec_elems(const Target& t, int nr) { return (size_t)nr * 3 * t.Npad; }

// Allocate (or reuse) a group's buffers for precision mode `prec`.
dda_status ensure_group(dda_ctx* c, Group& g, const Target& t, int prec, bool* realloc) {
    const int nr = g.nr;
    const size_t v64 = vec_elems(t, nr) * sizeof(Cx<double>);
    const int kp = (prec == DDA_SOLVE_FP32_REFINE) ? DDA_FP32 : DDA_FP64;
    const size_t vk = vec_elems(t, nr) * (kp == DDA_FP32 ? sizeof(Cx<float>) : sizeof(Cx<double>));
    unsigned before[24];
    int nb = 0;
    DevMem* all[] = {&g.b64, &g.x64, &g.r64, &g.slab32, &g.slab64, &g.kv[0], &g.kv[1], &g.kv[2], &g.kv[3],
                     &g.kv[4], &g.kv[5], &g.kv[6], &g.kv[7], &g.state, &g.active, &g.partials};
    for (DevMem* d : all) before[nb++] = d->gen;
    HCHK(c, g.waves.ensure(nr * sizeof(WaveDev)));
    HCHK(c, g.ainv64.ensure((size_t)nr * t.ncomp * sizeof(Cx<double>)));
    HCHK(c, g.ainv32.ensure((size_t)nr * t.ncomp * sizeof(Cx<float>)));
    HCHK(c, g.b64.ensure(v64));
    HCHK(c, g.x64.ensure(v64));
    HCHK(c, g.r64.ensure(v64));
    HCHK(c, g.slab64.ensure(slab_elems(t, nr) * sizeof(Cx<double>)));
    if (kp == DDA_FP32) HCHK(c, g.slab32.ensure(slab_elems(t, nr) * sizeof(Cx<float>)));
    for (int i = 0; i < 8; ++i) {
        if (g.kprec != kp) g.kv[i].release();
        HCHK(c, g.kv[i].ensure(vk));
    }
    g.kprec = kp;
    HCHK(c, g.state.ensure(nr * sizeof(BiState)));
    HCHK(c, g.active.ensure(nr * sizeof(int)));
    HCHK(c, g.mask.ensure(nr * sizeof(int)));
    HCHK(c, g.partials.ensure((size_t)nr * 4 * std::max(vec_blocks(t.Npad), 12 * t.n[0]) * 2 * sizeof(double)));
    HCHK(c, g.scale.ensure(nr * sizeof(double)));
    HCHK(c, g.tolrel2.ensure(nr * sizeof(double)));
    HCHK(c, g.maxit.ensure(nr * sizeof(int)));
    HCHK(c, g.norms.ensure(nr * sizeof(double)));
    nb = 0;
    bool changed = false;
    for (DevMem* d : all) changed |= (before[nb++] != d->gen);
    if (changed) {
        // zero the padded vectors once so that padding stays zero
        for (DevMem* d : {&g.b64, &g.x64, &g.r64}) HCHK(c, hipMemsetAsync(d->p, 0, d->n, c->stream));
        for (int i = 0; i < 8; ++i) HCHK(c, hipMemsetAsync(g.kv[i].p, 0, g.kv[i].n, c->stream));
    }
    *realloc = changed;
    return DDA_OK;
}


// One BiCGstab iteration for every group (precision T), enqueued on st.
template <class T>
hipError_t enqueue_iteration(dda_ctx* c, hipStream_t st, int k, const std::vector<char>& live) {
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        if (!live[gi]) continue;
        Group& g = *c->groups[gi];
        const Target& t = *c->tg[g.tgt];
        const int Np = t.Npad, nr = g.nr;
        Cx<T>* x = g.kv[0].as<Cx<T>>();
        Cx<T>* r = g.kv[1].as<Cx<T>>();
        Cx<T>* rh = g.kv[2].as<Cx<T>>();
        Cx<T>* v = g.kv[4].as<Cx<T>>();
        Cx<T>* s = g.kv[5].as<Cx<T>>();
        Cx<T>* tt = g.kv[6].as<Cx<T>>();
        // the direction vector alternates between two buffers so that the
        // fused update never reads what it writes; iteration parity picks them
        Cx<T>* pin = (k & 1) ? g.kv[7].as<Cx<T>>() : g.kv[3].as<Cx<T>>();
        Cx<T>* pout = (k & 1) ? g.kv[3].as<Cx<T>>() : g.kv[7].as<Cx<T>>();
        BiState* bs = g.state.as<BiState>();
        int* act = g.active.as<int>();
        double* part = g.partials.as<double>();
        hipError_t e;
        const bool fuse = (t.shape<T>().ct & 1) != 0 && !t.any_aniso;
        const int nbv = vec_blocks(Np), nbp = fuse ? 12 * t.n[0] : nbv;
        if (!fuse) pin = pout = g.kv[3].as<Cx<T>>();  // separate update kernel works in place
        if (fuse) {
            // one stream applies the previous iteration's pending x, r update
            // and forms the new direction (a separate kernel: in the forward
            // pass each of the four parity blocks of a plane would re-load all
            // five vectors); the inverse pass forms <rhat, v>
            if ((e = launch_bicg_upd<T>(Np, nr, x, r, pin, pout, v, rh, s, tt, bs, act, st)) != hipSuccess) return e;
            if ((e = matvec_group<T>(t, g, nr, pout, v, nullptr, act, MV_AX, st, MvDot{1, rh, part})) != hipSuccess)
                return e;
        } else {
            if ((e = launch_bicg_p<T>(Np, nr, pin, r, v, rh, bs, act, st)) != hipSuccess) return e;
            if ((e = matvec_group<T>(t, g, nr, pin, v, nullptr, act, MV_AX, st)) != hipSuccess) return e;
            if ((e = launch_dot<T>(Np, nr, 1, rh, v, nullptr, nullptr, part, act, st)) != hipSuccess) return e;
        }
        if (!fuse && (e = launch_scalars(0, nbp, nr, bs, part, act, 0, st)) != hipSuccess) return e;
        if (fuse) {
            // the inverse pass also forms <rhat, s>, <rhat, t> and ||s||^2, from
            // which the scalars follow without forming r = s - omega t; that
            // update is left pending for the next iteration's forward pass
            if ((e = matvec_group<T>(t, g, nr, s, tt, nullptr, act, MV_AX, st, MvDot{3, rh, part},
                                     MvUpd{2, r, v, s, bs, part})) !=
                hipSuccess)
                return e;
            if ((e = launch_scalars(3, nbp, nr, bs, part, act, k & 1, st)) != hipSuccess) return e;
            continue;
        } else {
            if ((e = launch_bicg_s<T>(Np, nr, s, r, v, bs, act, st)) != hipSuccess) return e;
            if ((e = matvec_group<T>(t, g, nr, s, tt, nullptr, act, MV_AX, st)) != hipSuccess) return e;
            if ((e = launch_dot<T>(Np, nr, 2, tt, s, tt, tt, part, act, st)) != hipSuccess) return e;
        }
        if ((e = launch_scalars(1, nbp, nr, bs, part, act, 0, st)) != hipSuccess) return e;
        if ((e = launch_bicg_xr<T>(Np, nr, x, r, pout, s, tt, rh, bs, part, act, st)) != hipSuccess) return e;
        if ((e = launch_scalars(2, nbv, nr, bs, part, act, 0, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// One BiCGstab(2) cycle (two BiCG steps, one minimal-residual step of
// degree 2; the guide's PBCGS2) for every live group (precision T).  With the
// specialised plane kernels the inner products of each matvec are formed by
// its inverse pass; otherwise by separate reductions in the same layout.
template <class T>
hipError_t enqueue_cycle_l2(dda_ctx* c, hipStream_t st, const std::vector<char>& live) {
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        if (!live[gi]) continue;
        Group& g = *c->groups[gi];
        const Target& t = *c->tg[g.tgt];
        const int Np = t.Npad, nr = g.nr;
        Cx<T>* x = g.kv[0].as<Cx<T>>();
        Cx<T>* r0 = g.kv[1].as<Cx<T>>();
        Cx<T>* rt = g.kv[2].as<Cx<T>>();
        Cx<T>* u0 = g.kv[3].as<Cx<T>>();
        Cx<T>* u1 = g.kv[4].as<Cx<T>>();
        Cx<T>* u2 = g.kv[5].as<Cx<T>>();
        Cx<T>* r1 = g.kv[6].as<Cx<T>>();
        Cx<T>* r2 = g.kv[7].as<Cx<T>>();
        BiState* bs = g.state.as<BiState>();
        int* act = g.active.as<int>();
        double* part = g.partials.as<double>();
        const bool fuse = (t.shape<T>().ct & 1) != 0 && !t.any_aniso;
        const int nbv = vec_blocks(Np), nbp = fuse ? 12 * t.n[0] : nbv;
        hipError_t e;
        auto mv_dot1 = [&](const Cx<T>* in, Cx<T>* out) -> hipError_t {
            // out = A in and <rt, out>
            if (fuse) return matvec_group<T>(t, g, nr, in, out, nullptr, act, MV_AX, st, MvDot{1, rt, part});
            hipError_t e2 = matvec_group<T>(t, g, nr, in, out, nullptr, act, MV_AX, st);
            if (e2 != hipSuccess) return e2;
            return launch_dot<T>(Np, nr, 1, rt, out, nullptr, nullptr, part, act, st);
        };
        if ((e = launch_l2_scalars(0, nbv, nr, bs, part, act, st)) != hipSuccess) return e;
        if ((e = launch_l2_update<T>(1, Np, nr, x, r0, rt, u0, u1, u2, r1, r2, bs, part, act, st)) != hipSuccess) return e;
        if ((e = mv_dot1(u0, u1)) != hipSuccess) return e;
        if ((e = launch_l2_scalars(1, nbp, nr, bs, part, act, st)) != hipSuccess) return e;
        if ((e = launch_l2_update<T>(2, Np, nr, x, r0, rt, u0, u1, u2, r1, r2, bs, part, act, st)) != hipSuccess) return e;
        if ((e = mv_dot1(r0, r1)) != hipSuccess) return e;
        if ((e = launch_l2_scalars(2, nbp, nr, bs, part, act, st)) != hipSuccess) return e;
        if ((e = launch_l2_update<T>(3, Np, nr, x, r0, rt, u0, u1, u2, r1, r2, bs, part, act, st)) != hipSuccess) return e;
        if ((e = mv_dot1(u1, u2)) != hipSuccess) return e;
        if ((e = launch_l2_scalars(1, nbp, nr, bs, part, act, st)) != hipSuccess) return e;
        if ((e = launch_l2_update<T>(4, Np, nr, x, r0, rt, u0, u1, u2, r1, r2, bs, part, act, st)) != hipSuccess) return e;
        // r2 = A r1 with the minimal-residual inner products of r0, r1, r2
        if (fuse) {
            if ((e = matvec_group<T>(t, g, nr, r1, r2, nullptr, act, MV_AX, st, MvDot{3, r0, part})) != hipSuccess)
                return e;
        } else {
            if ((e = matvec_group<T>(t, g, nr, r1, r2, nullptr, act, MV_AX, st)) != hipSuccess) return e;
            if ((e = launch_l2_mrdot<T>(Np, nr, r0, r1, r2, part, act, st)) != hipSuccess) return e;
        }
        if ((e = launch_l2_scalars(3, nbp, nr, bs, part, act, st)) != hipSuccess) return e;
        if ((e = launch_l2_update<T>(5, Np, nr, x, r0, rt, u0, u1, u2, r1, r2, bs, part, act, st)) != hipSuccess) return e;
        if ((e = launch_l2_scalars(4, nbv, nr, bs, part, act, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Inner BiCGstab on all groups: solves A d = b_inner from d = 0, where b_inner
// is already in kv[1] (r).  Per-rhs relative tolerance and iteration budget
// are in g.tolrel2 / g.maxit.  Returns when no rhs is active.
template <class T>
dda_status inner_solve(dda_ctx* c, int kiters, bool use_graph) {
    hipStream_t st = c->stream;
    for (auto& gp : c->groups) {
        Group& g = *gp;
        const Target& t = *c->tg[g.tgt];
        Cx<T>* x = g.kv[0].as<Cx<T>>();
        Cx<T>* r = g.kv[1].as<Cx<T>>();
        // b_inner currently in r: copy into x temporarily? use init kernel with b = r
        HCHK(c, launch_bicg_init<T>(t.Npad, g.nr, r, x, r, g.kv[2].as<Cx<T>>(), g.kv[3].as<Cx<T>>(),
                                    g.kv[4].as<Cx<T>>(), st));
        HCHK(c, launch_dot<T>(t.Npad, g.nr, 1, r, r, nullptr, nullptr, g.partials.as<double>(), nullptr, st));
        if (c->solver == DDA_SOLVER_BICGSTAB2)
            HCHK(c, launch_l2_state_init(t.Npad, g.nr, g.state.as<BiState>(), g.partials.as<double>(),
                                         g.tolrel2.as<double>(), g.maxit.as<int>(), g.active.as<int>(),
                                         c->force_restart, g.tcap > 0 ? g.trace.as<double>() : nullptr, g.tcap, st));
        else
            HCHK(c, launch_state_init(t.Npad, g.nr, g.state.as<BiState>(), g.partials.as<double>(),
                                      g.tolrel2.as<double>(), g.maxit.as<int>(), g.active.as<int>(), c->force_restart,
                                      g.tcap > 0 ? g.trace.as<double>() : nullptr, g.tcap, st));
    }
    const int prec = std::is_same<T, double>::value ? DDA_FP64 : DDA_FP32;
    if (c->gkey_gen != c->ws_gen || c->gkey_prec != prec || c->gkey_k != kiters || c->gkey_solver != c->solver) {
        c->drop_graphs();
        c->gkey_gen = c->ws_gen;
        c->gkey_prec = prec;
        c->gkey_k = kiters;
        c->gkey_solver = c->solver;
    }
    // one BiCGstab(2) cycle takes two BiCG steps: kiters / 2 cycles per replay
    auto enqueue = [&](int k, const std::vector<char>& lv) -> hipError_t {
        if (c->solver == DDA_SOLVER_BICGSTAB2) return (k & 1) ? hipSuccess : enqueue_cycle_l2<T>(c, st, lv);
        return enqueue_iteration<T>(c, st, k, lv);
    };
    // Replays run one ahead of the convergence poll: replay i + 1 is queued
    // before the flags left by replay i are read (pinned copies and events),
    // so the device does not idle between replays; the replay queued after
    // the last active rhs stopped runs with every block exiting early.
    const size_t ng = c->groups.size();
    std::vector<size_t> off(ng + 1, 0);
    for (size_t k = 0; k < ng; ++k) off[k + 1] = off[k] + c->groups[k]->nr;
    if (c->poll_cap < 2 * off[ng]) {
        if (c->poll_host) (void)hipHostFree(c->poll_host);
        c->poll_host = nullptr;
        c->poll_cap = 0;
        HCHK(c, hipHostMalloc((void**)&c->poll_host, 2 * off[ng] * sizeof(int), hipHostMallocDefault));
        c->poll_cap = 2 * off[ng];
    }
    for (auto& e : c->evpoll)
        if (!e) HCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    auto post_poll = [&](int slot) -> dda_status {
        for (size_t k = 0; k < ng; ++k)
            HCHK(c, hipMemcpyAsync(c->poll_host + slot * off[ng] + off[k], c->groups[k]->active.p,
                                   c->groups[k]->nr * sizeof(int), hipMemcpyDeviceToHost, st));
        HCHK(c, hipEventRecord(c->evpoll[slot], st));
        return DDA_OK;
    };
    auto read_poll = [&](int slot, std::vector<char>& lv) -> int {  // -1: HIP error, else any active
        if (hipEventSynchronize(c->evpoll[slot]) != hipSuccess) return -1;
        int any = 0;
        for (size_t k = 0; k < ng; ++k) {
            lv[k] = 0;
            for (size_t i = off[k]; i < off[k + 1]; ++i) lv[k] |= (c->poll_host[slot * off[ng] + i] != 0);
            any |= lv[k];
        }
        return any;
    };
    auto launch = [&](const std::vector<char>& lv) -> dda_status {
        if (use_graph) {
            auto it = c->gexec.find(lv);
            if (it == c->gexec.end()) {
                if (c->gexec.size() >= 32) c->drop_graphs();  // bound the cache over many live sets
                hipGraph_t graph;
                hipGraphExec_t ex = nullptr;
                HCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                hipError_t e = hipSuccess;
                for (int k = 0; k < kiters && e == hipSuccess; ++k) e = enqueue(k, lv);
                hipError_t e2 = hipStreamEndCapture(st, &graph);
                HCHK(c, e);
                HCHK(c, e2);
                e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                HCHK(c, e);
                it = c->gexec.emplace(lv, ex).first;
            }
            HCHK(c, hipGraphLaunch(it->second, st));
        } else {
            for (int k = 0; k < kiters; ++k) HCHK(c, enqueue(k, lv));
        }
        return DDA_OK;
    };
    // the first replay runs every group with a slot the refinement loop gave
    // an iteration budget (its mask); the state initialisation activates no
    // other slot, and one that starts converged only exits early
    std::vector<char> live(ng);
    int any = 0;
    for (size_t k = 0; k < ng; ++k) {
        live[k] = 0;
        for (int v : c->groups[k]->hmask) live[k] |= (v != 0);
        any |= live[k];
    }
    int slot = 0;
    if (any) {
        SCHK(launch(live));
        SCHK(post_poll(slot));
    }
    for (int guard = 0; any && guard < 1000000; ++guard) {
        SCHK(launch(live));  // one replay ahead of the flags being read
        SCHK(post_poll(slot ^ 1));
        any = read_poll(slot, live);
        if (any < 0) return fail(c, DDA_ERR_HIP, "inner solve: poll failed");
        slot ^= 1;
    }
    // apply the update the last fused iteration of every rhs left pending; the
    // direction of iteration k is in kv[7] for even k, kv[3] for odd k
    // (BiCGstab(2) applies every update within its cycle)
    for (auto& gp : c->groups) {
        if (c->solver == DDA_SOLVER_BICGSTAB2) break;
        Group& g = *gp;
        const Target& t = *c->tg[g.tgt];
        HCHK(c, launch_bicg_flush<T>(t.Npad, g.nr, g.kv[0].as<Cx<T>>(), g.kv[1].as<Cx<T>>(), g.kv[7].as<Cx<T>>(),
                                     g.kv[3].as<Cx<T>>(), g.kv[5].as<Cx<T>>(), g.kv[6].as<Cx<T>>(),
                                     g.state.as<BiState>(), st));
    }
    return DDA_OK;
}

// Keep the group's current solution, waves and 1/alpha in its history ring
// (depth 0 clears the ring).
dda_status push_history(dda_ctx* c, Group& g, const Target& t, int depth) {
    if (depth != g.hdepth) {
        g.hdepth = depth;
        g.hn = 0;
        g.hhead = 0;
    }
    if (depth == 0) return DDA_OK;
    hipStream_t st = c->stream;
    const int e = g.hhead;
    const size_t vb = vec_elems(t, g.nr) * sizeof(Cx<double>), ab = (size_t)g.nr * t.ncomp * sizeof(Cx<double>);
    HCHK(c, g.hx[e].ensure(vb));
    HCHK(c, g.hwv[e].ensure(g.nr * sizeof(WaveDev)));
    HCHK(c, g.hainvv[e].ensure(ab));
    HCHK(c, hipMemcpyAsync(g.hx[e].p, g.x64.p, vb, hipMemcpyDeviceToDevice, st));
    HCHK(c, hipMemcpyAsync(g.hwv[e].p, g.waves.p, g.nr * sizeof(WaveDev), hipMemcpyDeviceToDevice, st));
    HCHK(c, hipMemcpyAsync(g.hainvv[e].p, g.ainv64.p, ab, hipMemcpyDeviceToDevice, st));
    g.hhead = (e + 1) % depth;
    g.hn = std::min(g.hn + 1, depth);
    return DDA_OK;
}

// Solve the h x h normal equations G c = q (G Hermitian positive
// semi-definite, upper triangle given) by Gaussian elimination with partial
// pivoting after a relative diagonal shift of 1e-12.

// Least-squares guess over earlier solutions of the group's slots (the
// history ring, or only the previous solution held in x64 when the ring is
// empty): every solution is phase shifted to the current wave (as the
// PREV_SHIFT guess), multiplied by A in FP32, and the combination minimising
// ||E - A x|| per rhs becomes x64.  Its local field (1/alpha) x goes to g.esh,
// its residual field to g.rf and the residual's rms per site component to
// g.hrscale.
dda_status project_history(dda_ctx* c, Group& g, Target& t) {
    hipStream_t st = c->stream;
    const bool from_last = g.hn == 0;
    const int h = from_last ? 1 : g.hn, nr = g.nr;
    const size_t ve = vec_elems(t, nr);
    HCHK(c, g.pv32.ensure((size_t)HIST_MAX * ve * sizeof(Cx<float>)));
    const unsigned w_before = g.pw32.gen;
    HCHK(c, g.pw32.ensure((size_t)HIST_MAX * ve * sizeof(Cx<float>)));
    // the matvec writes the sites only: zero the padding of the products once
    if (g.pw32.gen != w_before) HCHK(c, hipMemsetAsync(g.pw32.p, 0, g.pw32.n, st));
    HCHK(c, g.slab32.ensure(slab_elems(t, nr) * sizeof(Cx<float>)));
    if (!t.have32) SCHK(ensure_green(c, t, DDA_FP32 | DDA_FP64));
    const int nblk = gram_blocks(t.Npad);
    HCHK(c, g.gpart.ensure((size_t)nr * nblk * HIST_NGRAM * 2 * sizeof(double)));
    HCHK(c, g.pcoef.ensure((size_t)nr * HIST_MAX * sizeof(Cx<double>)));
    Cx<float>* V = g.pv32.as<Cx<float>>();
    Cx<float>* W = g.pw32.as<Cx<float>>();
    HCHK(c, g.esh.ensure(ve * sizeof(Cx<float>)));
    HCHK(c, g.rf.ensure(ve * sizeof(Cx<float>)));
    HistSrc src{};
    src.h = h;
    for (int e = 0; e < h; ++e) {
        src.P[e] = from_last ? g.x64.as<Cx<double>>() : g.hx[e].as<Cx<double>>();
        src.ainv[e] = from_last ? g.ainvprev.as<Cx<double>>() : g.hainvv[e].as<Cx<double>>();
        src.w[e] = from_last ? g.wprev.as<WaveDev>() : g.hwv[e].as<WaveDev>();
    }
    HCHK(c, launch_prev_shift_hist(t.geo(), t.origin, nr, src, g.ainv64.as<Cx<double>>(), g.waves.as<WaveDev>(), V, ve,
                                   st));
    for (int e = 0; e < h; ++e)
        HCHK(c, matvec_group<float>(t, g, nr, V + e * ve, W + e * ve, nullptr, nullptr, MV_AX, st));
    // coefficients, combination, residual field and its norm on the device:
    // the guess takes no host round trip
    HCHK(c, launch_gram(t.Npad, nr, h, W, g.b64.as<Cx<double>>(), g.gpart.as<double>(), st));
    HCHK(c, launch_proj_coef(t.Npad, nr, h, g.gpart.as<double>(), g.pcoef.as<Cx<double>>(), st));
    HCHK(c, launch_hist_combine(t.geo(), nr, h, V, g.pcoef.as<Cx<double>>(), g.x64.as<Cx<double>>(),
                                g.ainv64.as<Cx<double>>(), g.esh.as<Cx<float>>(), W, g.b64.as<Cx<double>>(),
                                g.rf.as<Cx<float>>(), st));
    HCHK(c, g.rfn2.ensure(nr * sizeof(double)));
    HCHK(c, launch_norm2<float>(t.Npad, nr, g.rf.as<Cx<float>>(), g.partials.as<double>(), g.rfn2.as<double>(), st));
    g.has_r = true;
    return DDA_OK;
}

dda_status group_waves(dda_ctx* c, int nrhs, const dda_wave* waves) {
    // regroup only if the target pattern changed
    bool same = (int)c->rhs_group.size() == nrhs && c->last_nrhs == nrhs;
    if (same)
        for (int i = 0; i < nrhs; ++i)
            if (c->groups[c->rhs_group[i]]->tgt != waves[i].target) {
                same = false;
                break;
            }
    if (same) return DDA_OK;
    c->groups.clear();
    c->rhs_group.assign(nrhs, -1);
    c->rhs_slot.assign(nrhs, -1);
    for (int i = 0; i < nrhs; ++i) {
        int gi = -1;
        for (size_t k = 0; k < c->groups.size(); ++k)
            if (c->groups[k]->tgt == waves[i].target) gi = (int)k;
        if (gi < 0) {
            c->groups.emplace_back(new Group());
            gi = (int)c->groups.size() - 1;
            c->groups[gi]->tgt = waves[i].target;
        }
        Group& g = *c->groups[gi];
        c->rhs_group[i] = gi;
        c->rhs_slot[i] = g.nr++;
        g.idx.push_back(i);
    }
    c->last_nrhs = nrhs;
    c->ws_gen++;
    c->have_solution = false;
    return DDA_OK;
}

// error text of a failed dda_create (there is no context to hold it)
thread_local std::string g_create_err = "no error";

// Device scratch of dda_matvec_noalloc: one array per GPU for the life of
// the process.  Host code never passes its name to a kernel or a copy (on
// the host the name is only a stand-in for the symbol); it uses the device
// address that hipGetSymbolAddress returns for the current device, looked up
// once per device by dda_create and kept in g_scratch_ptr.
constexpr size_t NOALLOC_BYTES = (size_t)DDA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
constexpr int MAX_DEVICES = 64;
void* g_scratch_ptr[MAX_DEVICES] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on `device` (the current device); looked up on
// the first call per device.
hipError_t scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* dda_version(void) { return "dda-mi355x 0.1 (gfx950)"; }

dda_status dda_create(dda_ctx** out, int32_t device, void* hip_stream) {
    if (!out) return DDA_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return DDA_ERR_NO_DEVICE;
    if (device < 0 || device >= n) return DDA_ERR_INVALID_ARG;
    dda_ctx* c = new (std::nothrow) dda_ctx();
    if (!c) return DDA_ERR_OOM;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return DDA_ERR_HIP;
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return DDA_ERR_HIP;
        }
        c->own_stream = true;
    }
    hipError_t e1 = configure_fft_kernels(), e2 = configure_ct_kernels();
    void* sp = nullptr;
    if (e1 == hipSuccess && e2 == hipSuccess) e1 = scratch_address(device, &sp);
    if (e1 != hipSuccess || e2 != hipSuccess || hipEventCreate(&c->ev0) != hipSuccess ||
        hipEventCreate(&c->ev1) != hipSuccess) {
        g_create_err = std::string("dda_create: kernel configuration failed: ") +
                       hipGetErrorString(e1 != hipSuccess ? e1 : e2);
        delete c;
        return DDA_ERR_HIP;
    }
    *out = c;
    return DDA_OK;
}

dda_status dda_destroy(dda_ctx* c) {
    if (!c) return DDA_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    c->drop_graphs();
    c->groups.clear();
    c->tg.clear();
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    for (auto& e : c->evpoll)
        if (e) (void)hipEventDestroy(e);
    if (c->poll_host) (void)hipHostFree(c->poll_host);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return DDA_OK;
}

const char* dda_last_error(const dda_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

dda_status dda_add_target(dda_ctx* c, const int32_t dims[3], const uint8_t* occ, int32_t ncomp, const double* m,
                          double kd, int32_t alpha_kind, const double* origin, int32_t* id_out) {
    SCHK(check_ctx(c));
    std::unique_ptr<Target> t(new Target());
    dda_status s = build_target(c, *t, dims, occ, ncomp, m, kd, alpha_kind, origin);
    if (s < 0) return s;
    c->tg.push_back(std::move(t));
    if (id_out) *id_out = (int32_t)c->tg.size() - 1;
    c->groups.clear();
    c->rhs_group.clear();
    c->last_nrhs = 0;
    c->ws_gen++;
    c->have_solution = false;
    return s;
}

dda_status dda_set_target(dda_ctx* c, const int32_t dims[3], const uint8_t* occ, int32_t ncomp, const double* m,
                          double kd, int32_t alpha_kind, const double* origin) {
    SCHK(check_ctx(c));
    (void)hipStreamSynchronize(c->stream);
    c->groups.clear();
    c->tg.clear();
    return dda_add_target(c, dims, occ, ncomp, m, kd, alpha_kind, origin, nullptr);
}

dda_status dda_target_info(const dda_ctx* c, int32_t target, int64_t* n_sites, double* aeff) {
    if (!c || target < 0 || target >= (int)c->tg.size()) return DDA_ERR_INVALID_ARG;
    if (n_sites) *n_sites = c->tg[target]->N;
    if (aeff) *aeff = c->tg[target]->aeff;
    return DDA_OK;
}

dda_status dda_set_anisotropic(dda_ctx* c, int32_t target, int32_t comp, const double* m3, const double* angles) {
    SCHK(check_ctx(c));
    if (target < 0 || target >= (int)c->tg.size()) return fail(c, DDA_ERR_INVALID_ARG, "set_anisotropic: unknown target");
    Target& t = *c->tg[target];
    if (comp < 1 || comp > t.ncomp || !m3 || !angles)
        return fail(c, DDA_ERR_INVALID_ARG, "set_anisotropic: composition %d outside [1, %d] or null pointers", comp,
                    t.ncomp);
    for (int j = 0; j < 6; ++j)
        if (!std::isfinite(m3[j])) return fail(c, DDA_ERR_INVALID_ARG, "set_anisotropic: non-finite index");
    for (int j = 0; j < 3; ++j)
        if (!std::isfinite(angles[j])) return fail(c, DDA_ERR_INVALID_ARG, "set_anisotropic: non-finite angle");
    (void)hipStreamSynchronize(c->stream);
    const int q = comp - 1;
    double mkd = 0;
    for (int j = 0; j < 3; ++j) {
        t.m3[q][j] = cd(m3[2 * j], m3[2 * j + 1]);
        t.dfang[q][j] = angles[j];
        mkd = std::max(mkd, std::abs(t.m3[q][j]) * t.kd);
    }
    t.aniso[q] = 1;
    t.any_aniso = true;
    // the solve's groups, graphs and previous solutions refer to the old
    // diagonal: start over
    c->groups.clear();
    c->rhs_group.clear();
    c->last_nrhs = 0;
    c->ws_gen++;
    c->have_solution = false;
    if (mkd >= 1.0) {
        fail(c, DDA_WARN_MKD_GE_1, "|m| k d = %.3f >= 1 for composition %d", mkd, comp);
        return DDA_WARN_MKD_GE_1;
    }
    return DDA_OK;
}

dda_status dda_build_green_fft(dda_ctx* c, uint32_t prec) {
    SCHK(check_ctx(c));
    if (c->tg.empty()) return fail(c, DDA_ERR_STATE, "build_green_fft before set_target");
    if (!(prec & (DDA_FP32 | DDA_FP64))) return fail(c, DDA_ERR_INVALID_ARG, "prec must contain DDA_FP32 or DDA_FP64");
    for (auto& t : c->tg) SCHK(ensure_green(c, *t, prec | DDA_FP64));
    return DDA_OK;
}

dda_status dda_inverse_polarizability(const dda_ctx* c, int32_t target, const dda_wave* w, double* out) {
    if (!c || !w || !out || target < 0 || target >= (int)c->tg.size()) return DDA_ERR_INVALID_ARG;
    const Target& t = *c->tg[target];
    for (int i = 0; i < t.ncomp; ++i) {
        const cd a = inverse_alpha(t.m[i], t.kd, t.alpha_kind, w->khat, w->e0);
        out[2 * i] = a.real();
        out[2 * i + 1] = a.imag();
    }
    return DDA_OK;
}

namespace {

// Rows of the right-hand sides of group g from an ABI buffer ([nrhs][N][3]
// complex128 of all rhs of the call, each with its own target's N) into the
// device layout `out` ([nr][3][Npad], zero padding).  `tmp` is staging.
dda_status gather_abi_rows(dda_ctx* c, const Group& g, const Target& t, const dda_wave* waves, const void* src,
                           bool devptr, DevMem& tmp, Cx<double>* out, hipStream_t st) {
    const size_t per = (size_t)t.N * 3 * sizeof(Cx<double>);
    HCHK(c, tmp.ensure(per * g.nr));
    for (int s = 0; s < g.nr; ++s) {
        size_t off = 0;
        for (int q = 0; q < g.idx[s]; ++q) off += (size_t)c->tg[waves[q].target]->N * 3 * sizeof(Cx<double>);
        HCHK(c, hipMemcpyAsync((char*)tmp.p + s * per, (const char*)src + off, per,
                               devptr ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    }
    HCHK(c, launch_from_abi<double>(t.geo(), g.nr, tmp.as<Cx<double>>(), out, st));
    HCHK(c, hipStreamSynchronize(st));  // the staging is reused by the next group
    return DDA_OK;
}

// dda_solve and dda_solve_field: e_inc NULL generates the plane waves.
dda_status solve_impl(dda_ctx* c, int32_t nrhs, const dda_wave* waves, const dda_solve_opts* o, const void* e_inc,
                      const void* p0, void* p_out, dda_solve_stats* stats) {
    SCHK(check_ctx(c));
    if (nrhs <= 0 || !waves || !o) return fail(c, DDA_ERR_INVALID_ARG, "solve: nrhs <= 0 or null waves/opts");
    if (c->tg.empty()) return fail(c, DDA_ERR_STATE, "solve before set_target");
    for (int i = 0; i < nrhs; ++i) {
        if (waves[i].target < 0 || waves[i].target >= (int)c->tg.size())
            return fail(c, DDA_ERR_INVALID_ARG, "wave %d: unknown target %d", i, waves[i].target);
        double kn = 0;
        for (int j = 0; j < 3; ++j) kn += waves[i].khat[j] * waves[i].khat[j];
        if (std::fabs(kn - 1.0) > 1e-6) return fail(c, DDA_ERR_INVALID_ARG, "wave %d: |khat| != 1", i);
        // the efficiencies are normalised by |E0|^2 = 1 and LDR's S assumes it
        double en = 0;
        for (int j = 0; j < 6; ++j) en += waves[i].e0[j] * waves[i].e0[j];
        if (std::fabs(en - 1.0) > 1e-6) return fail(c, DDA_ERR_INVALID_ARG, "wave %d: |e0| != 1", i);
    }
    if (o && o->restart_every < 0) return fail(c, DDA_ERR_INVALID_ARG, "restart_every < 0");
    if (o && o->solver != DDA_SOLVER_BICGSTAB && o->solver != DDA_SOLVER_BICGSTAB2)
        return fail(c, DDA_ERR_INVALID_ARG, "unknown solver %d", o->solver);
    const double tol = o->tol > 0 ? o->tol : 1e-5;
    const int max_iter = o->max_iter > 0 ? o->max_iter : 1000;
    const int prec = o->prec;
    if (prec != DDA_SOLVE_FP64 && prec != DDA_SOLVE_FP32_REFINE) return fail(c, DDA_ERR_INVALID_ARG, "bad prec");
    const bool devptr = (o->flags & DDA_DEVICE_PTRS) != 0;
    const bool use_graph = !(o->flags & DDA_NO_GRAPH);
    c->force_restart = o->restart_every;
    c->solver = o->solver;
    {
        const char* tp = std::getenv("DDA_TRACE");
        c->trace_path = tp ? tp : "";
    }
    const bool tracing = !c->trace_path.empty();
    c->ncalls++;
    // an even count keeps the alternating direction buffers aligned across replays
    const int kiters = 2 * std::max(1, ((o->graph_iters > 0 ? o->graph_iters : 4) + 1) / 2);
    if (o->guess == DDA_GUESS_USER && !p0) return fail(c, DDA_ERR_INVALID_ARG, "GUESS_USER needs p0");
    if (o->guess < DDA_GUESS_ZERO || o->guess > DDA_GUESS_PROJECT)
        return fail(c, DDA_ERR_INVALID_ARG, "unknown guess %d", o->guess);
    if (o->history < 0 || o->history > HIST_MAX)
        return fail(c, DDA_ERR_INVALID_ARG, "history %d outside [0, %d]", o->history, HIST_MAX);
    if (o->guess == DDA_GUESS_NN && !c->nn) return fail(c, DDA_ERR_STATE, "no learned-guess model attached");
    // PREV, PREV_SHIFT and NN start from the previous solution of each slot
    const bool keep_prev = (o->guess == DDA_GUESS_PREV || o->guess == DDA_GUESS_PREV_SHIFT || o->guess == DDA_GUESS_NN ||
                            o->guess == DDA_GUESS_PROJECT);
    if (keep_prev && (!c->have_solution || c->last_nrhs != nrhs))
        return fail(c, DDA_ERR_STATE, "guess %d needs a previous solve with the same number of right-hand sides",
                    o->guess);
    if (o->guess == DDA_GUESS_PREV_SHIFT || o->guess == DDA_GUESS_PROJECT || o->guess == DDA_GUESS_NN)
        for (int i = 0; i < nrhs; ++i)
            if (c->tg[waves[i].target]->any_aniso)
                return fail(c, DDA_ERR_INVALID_ARG,
                            "guess %d carries local fields with a scalar 1/alpha: not for anisotropic targets", o->guess);
    if (!keep_prev) SCHK(group_waves(c, nrhs, waves));
    else
        for (int i = 0; i < nrhs; ++i)
            if (c->groups[c->rhs_group[i]]->tgt != waves[i].target)
                return fail(c, DDA_ERR_STATE, "GUESS_PREV: rhs %d changed target", i);
    hipStream_t st = c->stream;
    HCHK(c, hipEventRecord(c->ev0, st));
    // spectra and workspaces
    for (auto& gp : c->groups) {
        Target& t = *c->tg[gp->tgt];
        SCHK(ensure_green(c, t, DDA_FP64 | (prec == DDA_SOLVE_FP32_REFINE ? DDA_FP32 : 0)));
        bool re = false;
        SCHK(ensure_group(c, *gp, t, prec, &re));
        if (re) {
            c->ws_gen++;
            if (keep_prev) return fail(c, DDA_ERR_STATE, "GUESS_PREV: workspace changed");
        }
    }
    // per-iteration residual trace of the inner solves (DDA_TRACE)
    for (auto& gp : c->groups) {
        Group& g = *gp;
        g.tcap = tracing ? std::min(max_iter, 100000) : 0;
        if (tracing) HCHK(c, g.trace.ensure((size_t)g.nr * g.tcap * sizeof(double)));
    }
    FILE* tf = nullptr;
    if (tracing) {
        tf = std::fopen(c->trace_path.c_str(), "a");
        if (!tf) return fail(c, DDA_ERR_IO, "DDA_TRACE: cannot open %s", c->trace_path.c_str());
        std::fprintf(tf, "# solve call %lld: nrhs %d tol %g prec %s; columns: rhs outer iteration rel_resid kind\n",
                     c->ncalls, nrhs, tol, prec == DDA_SOLVE_FP64 ? "fp64" : "fp32_refine");
    }
    struct TraceCloser {
        FILE* f;
        ~TraceCloser() {
            if (f) std::fclose(f);
        }
    } trace_closer{tf};
    // keep the previous waves and polarizabilities of every slot
    for (auto& gp : c->groups) {
        Group& g = *gp;
        g.has_r = false;
        if (!keep_prev) continue;
        const Target& t = *c->tg[g.tgt];
        HCHK(c, g.wprev.ensure(g.nr * sizeof(WaveDev)));
        HCHK(c, g.ainvprev.ensure((size_t)g.nr * t.ncomp * sizeof(Cx<double>)));
        HCHK(c, hipMemcpyAsync(g.wprev.p, g.waves.p, g.nr * sizeof(WaveDev), hipMemcpyDeviceToDevice, st));
        HCHK(c, hipMemcpyAsync(g.ainvprev.p, g.ainv64.p, (size_t)g.nr * t.ncomp * sizeof(Cx<double>),
                               hipMemcpyDeviceToDevice, st));
    }
    // waves, polarizabilities, incident field, norms
    for (auto& gp : c->groups) {
        Group& g = *gp;
        Target& t = *c->tg[g.tgt];
        g.hw.resize(g.nr);
        g.hainv.resize((size_t)g.nr * t.ncomp);
        std::vector<Cx<float>>& a32 = g.hainv32;
        a32.resize(g.hainv.size());
        for (int s = 0; s < g.nr; ++s) {
            const dda_wave& w = waves[g.idx[s]];
            WaveDev& d = g.hw[s];
            for (int j = 0; j < 3; ++j) d.khat[j] = w.khat[j];
            for (int j = 0; j < 6; ++j) d.e[j] = w.e0[j];
            d.k = t.kd;
            d.pad = 0;
            for (int q = 0; q < t.ncomp; ++q) {
                const cd a = inverse_alpha(t.m[q], t.kd, t.alpha_kind, w.khat, w.e0);
                g.hainv[(size_t)s * t.ncomp + q] = a;
                a32[(size_t)s * t.ncomp + q] = Cx<float>{(float)a.real(), (float)a.imag()};
            }
        }
        if (t.any_aniso) {
            std::vector<dda_wave> ws(g.nr);
            for (int s = 0; s < g.nr; ++s) ws[s] = waves[g.idx[s]];
            aniso_tables(t, g, ws.data());
            HCHK(c, g.aten64.ensure(g.haten.size() * sizeof(cd)));
            HCHK(c, g.aten32.ensure(g.haten32.size() * sizeof(Cx<float>)));
            HCHK(c, hipMemcpyAsync(g.aten64.p, g.haten.data(), g.haten.size() * sizeof(cd), hipMemcpyHostToDevice, st));
            HCHK(c, hipMemcpyAsync(g.aten32.p, g.haten32.data(), g.haten32.size() * sizeof(Cx<float>),
                                   hipMemcpyHostToDevice, st));
        }
        HCHK(c, hipMemcpyAsync(g.waves.p, g.hw.data(), g.nr * sizeof(WaveDev), hipMemcpyHostToDevice, st));
        HCHK(c, hipMemcpyAsync(g.ainv64.p, g.hainv.data(), g.hainv.size() * sizeof(cd), hipMemcpyHostToDevice, st));
        HCHK(c, hipMemcpyAsync(g.ainv32.p, a32.data(), a32.size() * sizeof(Cx<float>), hipMemcpyHostToDevice, st));
    }
    // incident field: the plane waves, or the caller's field
    DevMem dtmp;
    for (auto& gp : c->groups) {
        Group& g = *gp;
        Target& t = *c->tg[g.tgt];
        if (e_inc) SCHK(gather_abi_rows(c, g, t, waves, e_inc, devptr, dtmp, g.b64.as<Cx<double>>(), st));
        else HCHK(c, launch_einc<double>(t.geo(), t.origin, g.waves.as<WaveDev>(), g.nr, g.b64.as<Cx<double>>(), st));
    }
    // initial guess
    for (auto& gp : c->groups) {
        Group& g = *gp;
        Target& t = *c->tg[g.tgt];
        if (o->guess == DDA_GUESS_ZERO) {
            HCHK(c, launch_fill<double>(g.x64.as<Cx<double>>(), vec_elems(t, g.nr), st));
        } else if (o->guess == DDA_GUESS_USER) {
            SCHK(gather_abi_rows(c, g, t, waves, p0, devptr, dtmp, g.x64.as<Cx<double>>(), st));
        }
        // PREV, PREV_SHIFT, NN: x64 holds the previous solution here
    }
    c->ms_guess = 0;
    if (keep_prev) {
        HCHK(c, hipEventRecord(c->ev1, st));
        for (auto& gp : c->groups) {
            Group& g = *gp;
            Target& t = *c->tg[g.tgt];
            g.has_r = false;
            // PREV keeps P_prev; PREV_SHIFT carries it to the new direction,
            // P0 = (1/alpha_prev) P_prev exp(i k (khat - khat_prev) . r) / (1/alpha);
            // PROJECT takes the least-squares combination of such shifted
            // solutions; NN corrects the PROJECT guess
            if (o->guess == DDA_GUESS_PREV_SHIFT)
                HCHK(c, launch_prev_shift(t.geo(), t.origin, g.nr, g.x64.as<Cx<double>>(), g.ainvprev.as<Cx<double>>(),
                                          g.ainv64.as<Cx<double>>(), g.wprev.as<WaveDev>(), g.waves.as<WaveDev>(),
                                          nullptr, g.x64.as<Cx<double>>(), nullptr, st));
            if (o->guess != DDA_GUESS_PROJECT && o->guess != DDA_GUESS_NN) continue;
            SCHK(project_history(c, g, t));
            if (o->guess != DDA_GUESS_NN) continue;
            std::vector<dda_wave> gw(g.nr);
            for (int s = 0; s < g.nr; ++s) gw[s] = waves[g.idx[s]];
            hipError_t e = nn_guess_group(c->nn, site_view(t), gw.data(), reinterpret_cast<const double*>(g.hainv.data()),
                                          g.nr, g.esh.as<Cx<float>>(), g.rf.as<Cx<float>>(), g.rfn2.as<double>(),
                                          g.x64.as<Cx<double>>(), st);
            if (e == hipErrorNotSupported)
                return fail(c, DDA_ERR_UNSUPPORTED_DIMS, "learned guess needs a cubic box with side divisible by 16");
            HCHK(c, e);
        }
        hipEvent_t eg;
        HCHK(c, hipEventCreate(&eg));
        HCHK(c, hipEventRecord(eg, st));
        HCHK(c, hipEventSynchronize(eg));
        float mg = 0;
        HCHK(c, hipEventElapsedTime(&mg, c->ev1, eg));
        (void)hipEventDestroy(eg);
        c->ms_guess = mg;
    }
    std::vector<double> bb(nrhs), rel(nrhs), grel(nrhs, 1.0);
    std::vector<int> done(nrhs, 0), iters(nrhs, 0), outer(nrhs, 0), mvs(nrhs, 0), stat(nrhs, 0);
    for (auto& gp : c->groups) {
        Group& g = *gp;
        Target& t = *c->tg[g.tgt];
        HCHK(c, launch_norm2<double>(t.Npad, g.nr, g.b64.as<Cx<double>>(), g.partials.as<double>(),
                                     g.norms.as<double>(), st));
        std::vector<double> h(g.nr);
        HCHK(c, hipMemcpyAsync(h.data(), g.norms.p, g.nr * sizeof(double), hipMemcpyDeviceToHost, st));
        HCHK(c, hipStreamSynchronize(st));
        for (int s = 0; s < g.nr; ++s) bb[g.idx[s]] = h[s];
    }
    for (int i = 0; i < nrhs; ++i)
        if (!std::isfinite(bb[i])) return fail(c, DDA_ERR_INVALID_ARG, "rhs %d: the incident field is not finite", i);
    const bool guessed = o->guess != DDA_GUESS_ZERO;
    float ms32 = 0, ms64 = 0;
    hipEvent_t e0 = c->ev0, ea, eb;
    HCHK(c, hipEventCreate(&ea));
    HCHK(c, hipEventCreate(&eb));
    const int max_outer = 40;
    for (int it_out = 0; it_out <= max_outer; ++it_out) {
        // FP64 residual r = b - A x for rhs not yet done; from x = 0 it is b
        // itself (copied, its norm is the one above), with no matvec
        const bool from_zero = it_out == 0 && !guessed;
        HCHK(c, hipEventRecord(ea, st));
        for (auto& gp : c->groups) {
            Group& g = *gp;
            Target& t = *c->tg[g.tgt];
            HCHK(c, g.hup.ensure(g.up_bytes()));
            int* mk = g.up_mask();
            for (int s = 0; s < g.nr; ++s) mk[s] = done[g.idx[s]] ? 0 : 1;
            HCHK(c, hipMemcpyAsync(g.mask.p, mk, g.nr * sizeof(int), hipMemcpyHostToDevice, st));
            if (from_zero) {
                HCHK(c, hipMemcpyAsync(g.r64.p, g.b64.p, vec_elems(t, g.nr) * sizeof(Cx<double>),
                                       hipMemcpyDeviceToDevice, st));
                continue;
            }
            HCHK(c, matvec_group<double>(t, g, g.nr, g.x64.as<Cx<double>>(), g.r64.as<Cx<double>>(),
                                         g.b64.as<Cx<double>>(), g.mask.as<int>(), MV_RESID, st));
            HCHK(c, launch_norm2<double>(t.Npad, g.nr, g.r64.as<Cx<double>>(), g.partials.as<double>(),
                                         g.norms.as<double>(), st));
        }
        HCHK(c, hipEventRecord(eb, st));
        HCHK(c, hipEventSynchronize(eb));
        float ms = 0;
        HCHK(c, hipEventElapsedTime(&ms, ea, eb));
        ms64 += ms;
        bool all_done = true;
        for (auto& gp : c->groups) {
            Group& g = *gp;
            Target& t = *c->tg[g.tgt];
            std::vector<double> h(g.nr);
            if (from_zero) {
                for (int s = 0; s < g.nr; ++s) h[s] = bb[g.idx[s]];
            } else {
                HCHK(c, hipMemcpy(h.data(), g.norms.p, g.nr * sizeof(double), hipMemcpyDeviceToHost));
            }
            // the residual mask's upload from g.hup has completed (event above)
            double* sc = g.up_scale();
            double* tr2 = g.up_tol2();
            int* mi = g.up_maxit();
            for (int s = 0; s < g.nr; ++s) {
                sc[s] = 1.0;
                tr2[s] = 0.0;
                mi[s] = 0;
            }
            for (int s = 0; s < g.nr; ++s) {
                const int i = g.idx[s];
                if (done[i]) continue;
                outer[i] += 1;
                if (!from_zero) mvs[i] += 1;
                double rr = h[s];
                double rl = bb[i] > 0 ? std::sqrt(rr / bb[i]) : 0.0;
                if (it_out == 0) {
                    if (guessed && !(rl <= 1.0) && !(o->flags & DDA_NO_FALLBACK)) {
                        // the guess is worse than P0 = 0 (or not finite): fall back to it
                        const size_t off = (size_t)s * 3 * t.Npad;
                        HCHK(c, launch_fill<double>(g.x64.as<Cx<double>>() + off, (size_t)3 * t.Npad, st));
                        HCHK(c, hipMemcpyAsync(g.r64.as<Cx<double>>() + off, g.b64.as<Cx<double>>() + off,
                                               (size_t)3 * t.Npad * sizeof(Cx<double>), hipMemcpyDeviceToDevice, st));
                        rr = bb[i];
                        rl = 1.0;
                    }
                    grel[i] = rl;
                }
                rel[i] = rl;
                if (tf) std::fprintf(tf, "%d %d %d %.9e fp64\n", i, outer[i], iters[i], rl);
                if (rl <= tol || bb[i] == 0) {
                    done[i] = 1;
                    continue;
                }
                if (!std::isfinite(rl)) {  // breakdown: no further refinement can help
                    done[i] = 1;
                    stat[i] = DDA_WARN_NOT_CONVERGED;
                    continue;
                }
                if (iters[i] >= max_iter || it_out == max_outer) {
                    done[i] = 1;
                    stat[i] = DDA_WARN_NOT_CONVERGED;
                    continue;
                }
                all_done = false;
                sc[s] = 1.0 / std::sqrt(rr);
                double tin;
                // inner target below the outer one by the drift the inner
                // recursive residual can have from the FP64 residual (FP32
                // vectors at 1e-5: well below a tenth of the tolerance); a
                // miss costs one short extra refinement
                if (prec == DDA_SOLVE_FP32_REFINE) tin = std::min(0.5, std::max(2e-6, 0.9 * tol / rl));
                else tin = std::min(0.5, std::max(1e-15, 0.9 * tol / rl));
                tr2[s] = tin * tin;
                mi[s] = max_iter - iters[i];
            }
            std::vector<int>& mk = g.hmask;
            mk.resize(g.nr);
            for (int s = 0; s < g.nr; ++s) mk[s] = g.up_mask()[s] = mi[s] > 0 ? 1 : 0;
        }
        if (all_done) break;
        // scale, tolerance, budget and mask of the inner solve: asynchronous
        // copies from pinned staging, ordered before it by the stream
        for (auto& gp : c->groups) {
            Group& g = *gp;
            HCHK(c, hipMemcpyAsync(g.scale.p, g.up_scale(), g.nr * sizeof(double), hipMemcpyHostToDevice, st));
            HCHK(c, hipMemcpyAsync(g.tolrel2.p, g.up_tol2(), g.nr * sizeof(double), hipMemcpyHostToDevice, st));
            HCHK(c, hipMemcpyAsync(g.maxit.p, g.up_maxit(), g.nr * sizeof(int), hipMemcpyHostToDevice, st));
            HCHK(c, hipMemcpyAsync(g.mask.p, g.up_mask(), g.nr * sizeof(int), hipMemcpyHostToDevice, st));
        }
        // inner solve: A d = r / ||r||
        HCHK(c, hipEventRecord(ea, st));
        for (auto& gp : c->groups) {
            Group& g = *gp;
            Target& t = *c->tg[g.tgt];
            if (prec == DDA_SOLVE_FP32_REFINE)
                HCHK(c, launch_demote(t.Npad, g.nr, g.r64.as<Cx<double>>(), g.kv[1].as<Cx<float>>(),
                                      g.scale.as<double>(), nullptr, st));
            else
                HCHK(c, hipMemcpyAsync(g.kv[1].p, g.r64.p, vec_elems(t, g.nr) * sizeof(Cx<double>),
                                       hipMemcpyDeviceToDevice, st));
        }
        if (prec == DDA_SOLVE_FP32_REFINE) SCHK(inner_solve<float>(c, kiters, use_graph));
        else SCHK(inner_solve<double>(c, kiters, use_graph));
        for (auto& gp : c->groups) {
            Group& g = *gp;
            Target& t = *c->tg[g.tgt];
            if (prec == DDA_SOLVE_FP32_REFINE)
                HCHK(c, launch_promote_add(t.Npad, g.nr, g.x64.as<Cx<double>>(), g.kv[0].as<Cx<float>>(),
                                           g.scale.as<double>(), g.mask.as<int>(), g.state.as<BiState>(), st));
            else
                HCHK(c, launch_axpy_masked<double>(t.Npad, g.nr, g.x64.as<Cx<double>>(), g.kv[0].as<Cx<double>>(),
                                                   g.mask.as<int>(), g.state.as<BiState>(), st));
            HCHK(c, g.hst.ensure(g.nr * sizeof(BiState)));
            HCHK(c, hipMemcpyAsync(g.hst.p, g.state.p, g.nr * sizeof(BiState), hipMemcpyDeviceToHost, st));
        }
        HCHK(c, hipEventRecord(eb, st));
        HCHK(c, hipEventSynchronize(eb));
        for (auto& gp : c->groups) {
            Group& g = *gp;
            const BiState* hs = g.hst.as<BiState>();
            const std::vector<int>& mk = g.hmask;
            std::vector<double> tr;
            if (tf) {
                tr.resize((size_t)g.nr * g.tcap);
                HCHK(c, hipMemcpy(tr.data(), g.trace.p, tr.size() * sizeof(double), hipMemcpyDeviceToHost));
            }
            for (int s = 0; s < g.nr; ++s) {
                if (!mk[s]) continue;
                const int i = g.idx[s];
                // the inner right-hand side is r / ||r|| (FP32 inner solves; its
                // recursive residual times the FP64 relative residual estimates
                // ||E - A P|| / ||E||) or r itself (FP64: divided by ||E||)
                const double tsc = prec == DDA_SOLVE_FP32_REFINE ? rel[i] : 1.0 / std::sqrt(bb[i]);
                if (tf)
                    for (int k = 0; k < std::min(hs[s].it, g.tcap); ++k)
                        std::fprintf(tf, "%d %d %d %.9e inner\n", i, outer[i], iters[i] + k + 1,
                                     tsc * std::sqrt(std::max(0.0, tr[(size_t)s * g.tcap + k])));
                iters[i] += hs[s].it;
                mvs[i] += 2 * hs[s].it;
                // a breakdown the inner solve could not recover from ended it
                // non-finite: its correction was not applied, and repeating
                // it from the same residual would end the same way
                if (!std::isfinite(hs[s].rr)) {
                    done[i] = 1;
                    stat[i] = DDA_WARN_NOT_CONVERGED;
                }
            }
        }
        HCHK(c, hipEventElapsedTime(&ms, ea, eb));
        if (prec == DDA_SOLVE_FP32_REFINE) ms32 += ms;
        else ms64 += ms;
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    // output
    if (p_out) {
        size_t off = 0;
        for (int i = 0; i < nrhs; ++i) {
            Group& g = *c->groups[c->rhs_group[i]];
            Target& t = *c->tg[g.tgt];
            const int s = c->rhs_slot[i];
            const size_t per = (size_t)t.N * 3 * sizeof(Cx<double>);
            HCHK(c, dtmp.ensure(per));
            HCHK(c, launch_to_abi<double>(t.geo(), 1, g.x64.as<Cx<double>>() + (size_t)s * 3 * t.Npad,
                                          devptr ? (Cx<double>*)((char*)p_out + off) : dtmp.as<Cx<double>>(), st));
            if (!devptr) HCHK(c, hipMemcpyAsync((char*)p_out + off, dtmp.p, per, hipMemcpyDeviceToHost, st));
            HCHK(c, hipStreamSynchronize(st));
            off += per;
        }
    }
    HCHK(c, hipEventRecord(c->ev1, st));
    HCHK(c, hipEventSynchronize(c->ev1));
    float mst = 0;
    HCHK(c, hipEventElapsedTime(&mst, e0, c->ev1));
    c->ms_mv32 = ms32;
    c->ms_mv64 = ms64;
    c->ms_total = mst;
    c->have_solution = true;
    c->last_waves.assign(waves, waves + nrhs);
    for (auto& gp : c->groups) SCHK(push_history(c, *gp, *c->tg[gp->tgt], o->history));
    int any_nc = 0;
    for (int i = 0; i < nrhs; ++i) {
        if (stats) {
            stats[i].iters = iters[i];
            stats[i].matvecs = mvs[i];
            stats[i].outer = outer[i];
            stats[i].status = stat[i];
            stats[i].rel_resid = rel[i];
            stats[i].guess_resid = grel[i];
        }
        any_nc |= stat[i] != 0;
    }
    if (any_nc) {
        fail(c, DDA_WARN_NOT_CONVERGED, "some right-hand sides did not reach tol=%g", tol);
        return DDA_WARN_NOT_CONVERGED;
    }
    return DDA_OK;
}

}  // namespace

dda_status dda_solve(dda_ctx* c, int32_t nrhs, const dda_wave* waves, const dda_solve_opts* o, const void* p0,
                     void* p_out, dda_solve_stats* stats) {
    return solve_impl(c, nrhs, waves, o, nullptr, p0, p_out, stats);
}

dda_status dda_solve_field(dda_ctx* c, int32_t nrhs, const dda_wave* waves, const dda_solve_opts* o,
                           const void* e_inc, const void* p0, void* p_out, dda_solve_stats* stats) {
    if (c && !e_inc) return fail(c, DDA_ERR_INVALID_ARG, "solve_field: null e_inc");
    return solve_impl(c, nrhs, waves, o, e_inc, p0, p_out, stats);
}

dda_status dda_matvec(dda_ctx* c, int32_t target, int32_t nrhs, const double* ainv, const void* x, void* y,
                      uint32_t prec, uint32_t flags) {
    SCHK(check_ctx(c));
    if (target < 0 || target >= (int)c->tg.size() || nrhs <= 0 || !x || !y)
        return fail(c, DDA_ERR_INVALID_ARG, "matvec: bad target/nrhs/pointers");
    if (prec != DDA_FP32 && prec != DDA_FP64) return fail(c, DDA_ERR_INVALID_ARG, "matvec: prec must be FP32 or FP64");
    Target& t = *c->tg[target];
    SCHK(ensure_green(c, t, prec | DDA_FP64));
    hipStream_t st = c->stream;
    Group g;
    g.tgt = target;
    g.nr = nrhs;
    std::vector<cd> ai((size_t)nrhs * t.ncomp);
    if (ainv) {
        for (size_t i = 0; i < ai.size(); ++i) ai[i] = cd(ainv[2 * i], ainv[2 * i + 1]);
    } else {
        const double kh[3] = {1, 0, 0}, e[6] = {0, 0, 1, 0, 0, 0};
        for (int s = 0; s < nrhs; ++s)
            for (int q = 0; q < t.ncomp; ++q) ai[(size_t)s * t.ncomp + q] = inverse_alpha(t.m[q], t.kd, t.alpha_kind, kh, e);
    }
    if (t.any_aniso) {
        // anisotropic compositions: the tensor of the target's prescription for
        // the wave khat = x, e0 = y (their entries of ainv are not used)
        std::vector<dda_wave> ws(nrhs);
        for (auto& w : ws) {
            w = dda_wave{};
            w.khat[0] = 1;
            w.e0[2] = 1;
        }
        g.hainv = ai;
        g.hainv32.resize(ai.size());
        aniso_tables(t, g, ws.data());
        ai = g.hainv;
        HCHK(c, g.aten64.ensure(g.haten.size() * sizeof(cd)));
        HCHK(c, g.aten32.ensure(g.haten32.size() * sizeof(Cx<float>)));
        HCHK(c, hipMemcpy(g.aten64.p, g.haten.data(), g.haten.size() * sizeof(cd), hipMemcpyHostToDevice));
        HCHK(c, hipMemcpy(g.aten32.p, g.haten32.data(), g.haten32.size() * sizeof(Cx<float>), hipMemcpyHostToDevice));
    }
    const size_t per = (size_t)t.N * 3 * sizeof(Cx<double>);
    DevMem dx, dy, vx, vy;
    HCHK(c, dx.ensure(per * nrhs));
    HCHK(c, dy.ensure(per * nrhs));
    const bool dev = flags & DDA_DEVICE_PTRS;
    HCHK(c, hipMemcpyAsync(dx.p, x, per * nrhs, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    if (prec == DDA_FP64) {
        HCHK(c, g.ainv64.ensure(ai.size() * sizeof(cd)));
        HCHK(c, hipMemcpyAsync(g.ainv64.p, ai.data(), ai.size() * sizeof(cd), hipMemcpyHostToDevice, st));
        HCHK(c, g.slab64.ensure(slab_elems(t, nrhs) * sizeof(Cx<double>)));
        HCHK(c, vx.ensure(vec_elems(t, nrhs) * sizeof(Cx<double>)));
        HCHK(c, vy.ensure(vec_elems(t, nrhs) * sizeof(Cx<double>)));
        HCHK(c, launch_from_abi<double>(t.geo(), nrhs, dx.as<Cx<double>>(), vx.as<Cx<double>>(), st));
        HCHK(c, matvec_group<double>(t, g, nrhs, vx.as<Cx<double>>(), vy.as<Cx<double>>(), nullptr, nullptr, MV_AX, st));
        HCHK(c, launch_to_abi<double>(t.geo(), nrhs, vy.as<Cx<double>>(), dy.as<Cx<double>>(), st));
    } else {
        std::vector<Cx<float>> a32(ai.size());
        for (size_t i = 0; i < ai.size(); ++i) a32[i] = Cx<float>{(float)ai[i].real(), (float)ai[i].imag()};
        HCHK(c, g.ainv32.ensure(a32.size() * sizeof(Cx<float>)));
        HCHK(c, hipMemcpyAsync(g.ainv32.p, a32.data(), a32.size() * sizeof(Cx<float>), hipMemcpyHostToDevice, st));
        HCHK(c, g.slab32.ensure(slab_elems(t, nrhs) * sizeof(Cx<float>)));
        HCHK(c, vx.ensure(vec_elems(t, nrhs) * sizeof(Cx<float>)));
        HCHK(c, vy.ensure(vec_elems(t, nrhs) * sizeof(Cx<float>)));
        HCHK(c, launch_from_abi<float>(t.geo(), nrhs, dx.as<Cx<double>>(), vx.as<Cx<float>>(), st));
        HCHK(c, matvec_group<float>(t, g, nrhs, vx.as<Cx<float>>(), vy.as<Cx<float>>(), nullptr, nullptr, MV_AX, st));
        HCHK(c, launch_to_abi<float>(t.geo(), nrhs, vy.as<Cx<float>>(), dy.as<Cx<double>>(), st));
    }
    HCHK(c, hipMemcpyAsync(y, dy.p, per * nrhs, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    HCHK(c, hipStreamSynchronize(st));
    return DDA_OK;
}

dda_status dda_matvec_noalloc(dda_ctx* c, int32_t target, int32_t nrhs, const void* ainv, const void* x, void* y,
                              uint32_t prec) {
    SCHK(check_ctx(c));
    if (target < 0 || target >= (int)c->tg.size() || nrhs <= 0 || !ainv || !x || !y)
        return fail(c, DDA_ERR_INVALID_ARG, "matvec_noalloc: bad target/nrhs/pointers");
    if (prec != DDA_FP32 && prec != DDA_FP64)
        return fail(c, DDA_ERR_INVALID_ARG, "matvec_noalloc: prec must be FP32 or FP64");
    Target& t = *c->tg[target];
    if (!(prec == DDA_FP32 ? t.have32 : t.have64))
        return fail(c, DDA_ERR_STATE, "matvec_noalloc: build the target's spectrum first (dda_build_green_fft)");
    const size_t esz = prec == DDA_FP32 ? sizeof(Cx<float>) : sizeof(Cx<double>);
    const size_t b_ainv = prec == DDA_FP32 ? align256((size_t)nrhs * t.ncomp * sizeof(Cx<float>)) : 0;
    const size_t b_vec = align256(vec_elems(t, nrhs) * esz);
    const size_t b_slab = align256(slab_elems(t, nrhs) * esz);
    const size_t need = b_ainv + 2 * b_vec + b_slab;
    if (need > NOALLOC_BYTES)
        return fail(c, DDA_ERR_INVALID_ARG, "matvec_noalloc: %d rhs of this target need %zu bytes of scratch, above the "
                    "%zu-byte limit (use fewer rhs or dda_matvec)", nrhs, need, NOALLOC_BYTES);
    void* base = nullptr;
    {
        // looked up by dda_create on this context's device
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = c->device < MAX_DEVICES ? g_scratch_ptr[c->device] : nullptr;
    }
    if (!base) return fail(c, DDA_ERR_STATE, "matvec_noalloc: no scratch address for device %d", c->device);
    unsigned char* p = static_cast<unsigned char*>(base);
    hipStream_t st = c->stream;
    const Geo g = t.geo();
    const Cx<double>* xin = static_cast<const Cx<double>*>(x);
    Cx<double>* yout = static_cast<Cx<double>*>(y);
    if (prec == DDA_FP64) {
        Cx<double>* vx = reinterpret_cast<Cx<double>*>(p);
        Cx<double>* vy = reinterpret_cast<Cx<double>*>(p + b_vec);
        Cx<double>* slab = reinterpret_cast<Cx<double>*>(p + 2 * b_vec);
        HCHK(c, launch_from_abi<double>(g, nrhs, xin, vx, st));
        HCHK(c, launch_matvec<double>(g, t.tw<double>(), t.plans, t.shape<double>(), nrhs, vx, vy, nullptr, slab,
                                      t.ghat_for<double>(t.shape<double>()), static_cast<const Cx<double>*>(ainv),
                                      nullptr, MV_AX, st));
        HCHK(c, launch_to_abi<double>(g, nrhs, vy, yout, st));
    } else {
        Cx<float>* a32 = reinterpret_cast<Cx<float>*>(p);
        Cx<float>* vx = reinterpret_cast<Cx<float>*>(p + b_ainv);
        Cx<float>* vy = reinterpret_cast<Cx<float>*>(p + b_ainv + b_vec);
        Cx<float>* slab = reinterpret_cast<Cx<float>*>(p + b_ainv + 2 * b_vec);
        HCHK(c, launch_demote_table(nrhs * t.ncomp, static_cast<const Cx<double>*>(ainv), a32, st));
        HCHK(c, launch_from_abi<float>(g, nrhs, xin, vx, st));
        HCHK(c, launch_matvec<float>(g, t.tw<float>(), t.plans, t.shape<float>(), nrhs, vx, vy, nullptr, slab,
                                     t.ghat_for<float>(t.shape<float>()), a32, nullptr, MV_AX, st));
        HCHK(c, launch_to_abi<float>(g, nrhs, vy, yout, st));
    }
    return DDA_OK;
}

}  // extern "C"

namespace {

// The tensor part of the absorption sums of an anisotropic target's group,
// added to h[3 s + 1] (the layout of launch_xsec's output) after the stream
// has run; synchronizes the stream.
dda_status add_aniso_abs(dda_ctx* c, Group& g, const Target& t, double* h, hipStream_t st) {
    if (!t.any_aniso) return DDA_OK;
    DevMem& d = c->scr[7];
    HCHK(c, d.ensure(g.nr * sizeof(double)));
    HCHK(c, launch_aniso_abs(t.geo(), g.nr, g.x64.as<Cx<double>>(), g.aten64.as<Cx<double>>(), g.partials.as<double>(),
                             d.as<double>(), st));
    std::vector<double> a(g.nr);
    HCHK(c, hipMemcpyAsync(a.data(), d.p, g.nr * sizeof(double), hipMemcpyDeviceToHost, st));
    HCHK(c, hipStreamSynchronize(st));
    for (int s = 0; s < g.nr; ++s) h[3 * s + 1] += a[s];
    return DDA_OK;
}

}  // namespace

extern "C" {

dda_status dda_cross_sections(dda_ctx* c, int32_t nrhs, double* q) {
    SCHK(check_ctx(c));
    if (!c->have_solution) return fail(c, DDA_ERR_STATE, "cross_sections before a solve");
    if (nrhs != c->last_nrhs || !q) return fail(c, DDA_ERR_INVALID_ARG, "cross_sections: nrhs must match the last solve");
    hipStream_t st = c->stream;
    DevMem& out = c->scr[0];
    for (auto& gp : c->groups) {
        Group& g = *gp;
        Target& t = *c->tg[g.tgt];
        HCHK(c, out.ensure(3 * g.nr * sizeof(double)));
        HCHK(c, launch_xsec(t.geo(), g.nr, g.b64.as<Cx<double>>(), g.x64.as<Cx<double>>(), g.ainv64.as<Cx<double>>(),
                            t.kd * t.kd * t.kd, g.partials.as<double>(), out.as<double>(), st));
        std::vector<double> h(3 * g.nr);
        HCHK(c, hipMemcpyAsync(h.data(), out.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        SCHK(add_aniso_abs(c, g, t, h.data(), st));
        HCHK(c, hipStreamSynchronize(st));
        const double area = PI * t.aeff * t.aeff;
        for (int s = 0; s < g.nr; ++s) {
            const int i = g.idx[s];
            const double qext = 4 * PI * t.kd * h[3 * s] / area, qabs = 4 * PI * t.kd * h[3 * s + 1] / area;
            q[3 * i] = qext;
            q[3 * i + 1] = qabs;
            q[3 * i + 2] = qext - qabs;
        }
    }
    return DDA_OK;
}

dda_status dda_cross_sections_phi(dda_ctx* c, int32_t npairs, int32_t ncomb, const double* coeffs, double* q) {
    SCHK(check_ctx(c));
    if (!c->have_solution) return fail(c, DDA_ERR_STATE, "cross_sections_phi before a solve");
    if (npairs < 1 || ncomb < 1 || !coeffs || !q || 2 * npairs != c->last_nrhs)
        return fail(c, DDA_ERR_INVALID_ARG, "cross_sections_phi: need 2 * npairs == rhs of the last solve");
    for (auto& gp : c->groups)
        if (c->tg[gp->tgt]->any_aniso)
            return fail(c, DDA_ERR_INVALID_ARG, "cross_sections_phi: not for anisotropic targets");
    for (int p = 0; p < npairs; ++p) {
        const int i0 = 2 * p, i1 = 2 * p + 1;
        if (c->rhs_group[i0] != c->rhs_group[i1])
            return fail(c, DDA_ERR_INVALID_ARG, "cross_sections_phi: pair %d spans two targets", p);
        const dda_wave &w0 = c->last_waves[i0], &w1 = c->last_waves[i1];
        for (int k = 0; k < 3; ++k)
            if (std::abs(w0.khat[k] - w1.khat[k]) > 1e-12)
                return fail(c, DDA_ERR_INVALID_ARG, "cross_sections_phi: pair %d has two incidence directions", p);
        const Target& t = *c->tg[c->groups[c->rhs_group[i0]]->tgt];
        if (t.alpha_kind == DDA_ALPHA_LDR)
            return fail(c, DDA_ERR_INVALID_ARG,
                        "cross_sections_phi: the LDR polarizability depends on the polarization, so combinations "
                        "of solutions are not solutions");
    }
    hipStream_t st = c->stream;
    DevMem &dslots = c->scr[0], &dpart = c->scr[1];
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        Group& g = *c->groups[gi];
        const Target& t = *c->tg[g.tgt];
        std::vector<int> pairs, slots;
        for (int p = 0; p < npairs; ++p)
            if (c->rhs_group[2 * p] == (int)gi) {
                pairs.push_back(p);
                slots.push_back(c->rhs_slot[2 * p]);
                slots.push_back(c->rhs_slot[2 * p + 1]);
            }
        if (pairs.empty()) continue;
        const int np = (int)pairs.size(), nblk = xsec_pair_blocks(t.N);
        HCHK(c, dslots.ensure(slots.size() * sizeof(int)));
        HCHK(c, dpart.ensure((size_t)np * nblk * 16 * sizeof(double)));
        HCHK(c, hipMemcpyAsync(dslots.p, slots.data(), slots.size() * sizeof(int), hipMemcpyHostToDevice, st));
        HCHK(c, launch_xsec_pair(t.geo(), np, g.b64.as<Cx<double>>(), g.x64.as<Cx<double>>(),
                                 g.ainv64.as<Cx<double>>(), t.kd * t.kd * t.kd, dslots.as<int>(), dpart.as<double>(),
                                 st));
        std::vector<double> h((size_t)np * nblk * 16);
        HCHK(c, hipMemcpyAsync(h.data(), dpart.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HCHK(c, hipStreamSynchronize(st));
        const double scale = 4 * PI * t.kd / (PI * t.aeff * t.aeff);
        for (int k = 0; k < np; ++k) {
            double v[16] = {0};
            for (int b = 0; b < nblk; ++b)
                for (int e = 0; e < 16; ++e) v[e] += h[((size_t)k * nblk + b) * 16 + e];
            cd S[2][2], G[2][2];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    S[a][b] = cd(v[2 * (2 * a + b)], v[2 * (2 * a + b) + 1]);
                    G[a][b] = cd(v[8 + 2 * (2 * a + b)], v[9 + 2 * (2 * a + b)]);
                }
            const int p = pairs[k];
            for (int m = 0; m < ncomb; ++m)
                for (int l = 0; l < 2; ++l) {
                    const double* cc = coeffs + (((size_t)p * ncomb + m) * 2 + l) * 4;
                    const cd cl[2] = {cd(cc[0], cc[1]), cd(cc[2], cc[3])};
                    cd ext = 0, ab = 0;
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b) {
                            ext += std::conj(cl[a]) * cl[b] * S[a][b];
                            ab += std::conj(cl[a]) * cl[b] * G[a][b];
                        }
                    double* o = q + (((size_t)p * ncomb + m) * 2 + l) * 3;
                    o[0] = scale * ext.imag();
                    o[1] = scale * ab.real();
                    o[2] = o[0] - o[1];
                }
        }
    }
    return DDA_OK;
}

dda_status dda_scattering_moments(dda_ctx* c, int32_t nrhs, int32_t ndir, const double* n_tf, const double* w,
                                  double* out) {
    SCHK(check_ctx(c));
    if (!c->have_solution) return fail(c, DDA_ERR_STATE, "scattering_moments before a solve");
    if (nrhs != c->last_nrhs || ndir < 1 || !n_tf || !w || !out)
        return fail(c, DDA_ERR_INVALID_ARG, "scattering_moments: bad arguments (nrhs must match the last solve)");
    hipStream_t st = c->stream;
    DevMem &dn = c->scr[0], &dF = c->scr[1], &dP = c->scr[2], &dx = c->scr[3], &db = c->scr[4];
    HCHK(c, dn.ensure((size_t)ndir * 3 * sizeof(double)));
    HCHK(c, hipMemcpyAsync(dn.p, n_tf, (size_t)ndir * 3 * sizeof(double), hipMemcpyHostToDevice, st));
    for (auto& gp : c->groups) {
        Group& g = *gp;
        const Target& t = *c->tg[g.tgt];
        const Geo geo = t.geo();
        const double k = t.kd, k4 = k * k * k * k, area = PI * t.aeff * t.aeff;
        // Q_ext, Q_abs and Re sum E^* . P
        HCHK(c, dx.ensure(3 * g.nr * sizeof(double)));
        HCHK(c, launch_xsec(geo, g.nr, g.b64.as<Cx<double>>(), g.x64.as<Cx<double>>(), g.ainv64.as<Cx<double>>(),
                            k * k * k, g.partials.as<double>(), dx.as<double>(), st));
        // F(n) = sum_j P_j exp(-i k n . r_j) at the quadrature directions
        HCHK(c, dF.ensure((size_t)g.nr * ndir * 3 * sizeof(Cx<double>)));
        HCHK(c, dP.ensure((size_t)ampl_chunks(ndir, g.nr, t.N) * g.nr * ndir * 6 * sizeof(double)));
        HCHK(c, launch_ampl(geo, t.origin, k, g.nr, g.x64.as<Cx<double>>(), ndir, dn.as<double>(), dF.as<Cx<double>>(),
                            dP.as<double>(), st));
        std::vector<double> hx(3 * g.nr);
        std::vector<cd> F((size_t)g.nr * ndir * 3);
        HCHK(c, hipMemcpyAsync(hx.data(), dx.p, hx.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        SCHK(add_aniso_abs(c, g, t, hx.data(), st));
        HCHK(c, hipMemcpyAsync(F.data(), dF.p, F.size() * sizeof(cd), hipMemcpyDeviceToHost, st));
        // the backscattering direction -khat of each rhs
        std::vector<double> nb(3 * g.nr);
        for (int s2 = 0; s2 < g.nr; ++s2)
            for (int i = 0; i < 3; ++i) nb[3 * s2 + i] = -c->last_waves[g.idx[s2]].khat[i];
        HCHK(c, db.ensure(nb.size() * sizeof(double)));
        HCHK(c, hipMemcpyAsync(db.p, nb.data(), nb.size() * sizeof(double), hipMemcpyHostToDevice, st));
        std::vector<cd> Fb(3 * g.nr);
        DevMem &dFb = c->scr[5], &dPb = c->scr[6];
        HCHK(c, dFb.ensure(3 * sizeof(Cx<double>) * g.nr));
        HCHK(c, dPb.ensure((size_t)ampl_chunks(1, 1, t.N) * 6 * sizeof(double)));
        for (int s2 = 0; s2 < g.nr; ++s2)
            HCHK(c, launch_ampl(geo, t.origin, k, 1, g.x64.as<Cx<double>>() + (size_t)s2 * 3 * t.Npad, 1,
                                db.as<double>() + 3 * s2, dFb.as<Cx<double>>() + 3 * s2, dPb.as<double>(), st));
        HCHK(c, hipMemcpyAsync(Fb.data(), dFb.p, Fb.size() * sizeof(cd), hipMemcpyDeviceToHost, st));
        HCHK(c, hipStreamSynchronize(st));
        auto dcs = [&](const cd* f, const double* n) {  // k^4 |F - n (n . F)|^2
            const cd nf = n[0] * f[0] + n[1] * f[1] + n[2] * f[2];
            double a = 0;
            for (int i = 0; i < 3; ++i) a += std::norm(f[i] - n[i] * nf);
            return k4 * a;
        };
        for (int s2 = 0; s2 < g.nr; ++s2) {
            const double* kh = c->last_waves[g.idx[s2]].khat;
            const double qext = 4 * PI * k * hx[3 * s2] / area, qabs = 4 * PI * k * hx[3 * s2 + 1] / area;
            const double qsca = qext - qabs;
            double csum = 0, gv[3] = {0, 0, 0}, c2 = 0;
            for (int d = 0; d < ndir; ++d) {
                const double* n = n_tf + 3 * d;
                const double v = w[d] * dcs(&F[((size_t)s2 * ndir + d) * 3], n);
                const double ct = n[0] * kh[0] + n[1] * kh[1] + n[2] * kh[2];
                csum += v;
                for (int i = 0; i < 3; ++i) gv[i] += v * n[i];
                c2 += v * ct * ct;
            }
            double* o = out + (size_t)g.idx[s2] * DDA_NMOMENTS;
            o[0] = 2 * PI * k * hx[3 * s2 + 2] / area;  // Q_pha
            o[1] = dcs(&Fb[3 * s2], nb.data() + 3 * s2) / area;  // Q_bk
            o[2] = csum / area;  // Q_sca by the quadrature
            for (int i = 0; i < 3; ++i) o[3 + i] = gv[i] / area;  // Q_sca g
            o[6] = (gv[0] * kh[0] + gv[1] * kh[1] + gv[2] * kh[2]) / area / qsca;
            o[7] = c2 / area / qsca;
            for (int i = 0; i < 3; ++i) o[8 + i] = qext * kh[i] - o[3 + i];  // Q_pr
        }
    }
    return DDA_OK;
}

}  // extern "C"

namespace {
// Amplitudes of the last solve for directions shared by every rhs
// (per_rhs = false, n_tf: ndir x 3) or per rhs (n_tf: nrhs x ndir x 3,
// e_tf: nrhs x ndir x 6, rhs i taking block i).
dda_status amplitudes_impl(dda_ctx* c, int32_t nrhs, int32_t ndir, const double* n_tf, const double* e_tf, double* f,
                           bool per_rhs) {
    SCHK(check_ctx(c));
    if (!c->have_solution) return fail(c, DDA_ERR_STATE, "amplitudes before a solve");
    if (nrhs != c->last_nrhs || ndir <= 0 || !n_tf || !e_tf || !f)
        return fail(c, DDA_ERR_INVALID_ARG, "amplitudes: bad arguments (nrhs must match the last solve)");
    hipStream_t st = c->stream;
    DevMem &dn = c->scr[0], &dF = c->scr[1], &dP = c->scr[2], &dS = c->scr[3];
    const size_t nset = per_rhs ? (size_t)nrhs : 1;
    HCHK(c, dn.ensure(nset * ndir * 3 * sizeof(double)));
    HCHK(c, hipMemcpyAsync(dn.p, n_tf, nset * ndir * 3 * sizeof(double), hipMemcpyHostToDevice, st));
    for (auto& gp : c->groups) {
        Group& g = *gp;
        Target& t = *c->tg[g.tgt];
        HCHK(c, dF.ensure((size_t)g.nr * ndir * 3 * sizeof(Cx<double>)));
        HCHK(c, dP.ensure((size_t)ampl_chunks(ndir, g.nr, t.N) * g.nr * ndir * 6 * sizeof(double)));
        const int* dset = nullptr;
        if (per_rhs) {
            // direction block of each slot: its call-level rhs index
            HCHK(c, dS.ensure((size_t)g.nr * sizeof(int)));
            HCHK(c, hipMemcpyAsync(dS.p, g.idx.data(), (size_t)g.nr * sizeof(int), hipMemcpyHostToDevice, st));
            dset = dS.as<int>();
        }
        HCHK(c, launch_ampl(t.geo(), t.origin, t.kd, g.nr, g.x64.as<Cx<double>>(), ndir, dn.as<double>(),
                            dF.as<Cx<double>>(), dP.as<double>(), st, dset));
        std::vector<cd> F((size_t)g.nr * ndir * 3);
        HCHK(c, hipMemcpyAsync(F.data(), dF.p, F.size() * sizeof(cd), hipMemcpyDeviceToHost, st));
        HCHK(c, hipStreamSynchronize(st));
        const double k3 = t.kd * t.kd * t.kd;
        for (int s = 0; s < g.nr; ++s) {
            const int i = g.idx[s];
            const double* es = per_rhs ? e_tf + (size_t)i * ndir * 6 : e_tf;
            for (int d = 0; d < ndir; ++d) {
                const cd* Fv = &F[((size_t)s * ndir + d) * 3];
                for (int mm = 0; mm < 2; ++mm) {
                    const double* e = es + (size_t)d * 6 + 3 * mm;
                    const cd v = k3 * (e[0] * Fv[0] + e[1] * Fv[1] + e[2] * Fv[2]);
                    f[(((size_t)i * ndir + d) * 2 + mm) * 2] = v.real();
                    f[(((size_t)i * ndir + d) * 2 + mm) * 2 + 1] = v.imag();
                }
            }
        }
    }
    return DDA_OK;
}
}  // namespace

extern "C" {

dda_status dda_amplitudes(dda_ctx* c, int32_t nrhs, int32_t ndir, const double* n_tf, const double* e_tf, double* f) {
    return amplitudes_impl(c, nrhs, ndir, n_tf, e_tf, f, false);
}

dda_status dda_amplitudes_per_rhs(dda_ctx* c, int32_t nrhs, int32_t ndir, const double* n_tf, const double* e_tf,
                                  double* f) {
    return amplitudes_impl(c, nrhs, ndir, n_tf, e_tf, f, true);
}

dda_status dda_near_field(dda_ctx* c, int32_t nrhs, int32_t npts, const double* pts, double* E, double* B) {
    SCHK(check_ctx(c));
    if (!c->have_solution) return fail(c, DDA_ERR_STATE, "near_field before a solve");
    if (nrhs != c->last_nrhs || npts <= 0 || !pts || !E)
        return fail(c, DDA_ERR_INVALID_ARG, "near_field: bad arguments (nrhs must match the last solve)");
    hipStream_t st = c->stream;
    DevMem &dq = c->scr[0], &dout = c->scr[1];
    HCHK(c, dq.ensure((size_t)npts * 3 * sizeof(double)));
    HCHK(c, hipMemcpyAsync(dq.p, pts, (size_t)npts * 3 * sizeof(double), hipMemcpyHostToDevice, st));
    for (auto& gp : c->groups) {
        Group& g = *gp;
        const Target& t = *c->tg[g.tgt];
        const size_t per = (size_t)npts * 12;
        HCHK(c, dout.ensure(per * g.nr * sizeof(double)));
        HCHK(c, launch_near_field(t.geo(), t.origin, g.nr, g.x64.as<Cx<double>>(), g.waves.as<WaveDev>(),
                                  dq.as<double>(), npts, dout.as<double>(), st));
        std::vector<double> h(per * g.nr);
        HCHK(c, hipMemcpyAsync(h.data(), dout.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HCHK(c, hipStreamSynchronize(st));
        for (int s = 0; s < g.nr; ++s) {
            const size_t dst = (size_t)g.idx[s] * npts * 6;
            for (int q = 0; q < npts; ++q)
                for (int v = 0; v < 6; ++v) {
                    E[dst + (size_t)q * 6 + v] = h[((size_t)s * npts + q) * 12 + v];
                    if (B) B[dst + (size_t)q * 6 + v] = h[((size_t)s * npts + q) * 12 + 6 + v];
                }
        }
    }
    return DDA_OK;
}

dda_status dda_mueller(int32_t ndir, const double* f, const double* phi, const double* e01, const double* e02,
                       double* S, double* mu) {
    if (ndir <= 0 || !f || !phi || !e01 || !e02) return DDA_ERR_INVALID_ARG;
    const cd I(0, 1);
    const cd a = std::conj(cd(e01[2], e01[3])), b = std::conj(cd(e01[4], e01[5]));
    const cd cc = std::conj(cd(e02[2], e02[3])), d = std::conj(cd(e02[4], e02[5]));
    for (int k = 0; k < ndir; ++k) {
        const double* fk = f + (size_t)k * 8;
        const cd f11(fk[0], fk[1]), f12(fk[2], fk[3]), f21(fk[4], fk[5]), f22(fk[6], fk[7]);
        const double cp = std::cos(phi[k]), sp = std::sin(phi[k]);
        const cd S1 = -I * (f21 * (b * cp - a * sp) + f22 * (d * cp - cc * sp));
        const cd S2 = -I * (f11 * (a * cp + b * sp) + f12 * (cc * cp + d * sp));
        const cd S3 = I * (f11 * (b * cp - a * sp) + f12 * (d * cp - cc * sp));
        const cd S4 = I * (f21 * (a * cp + b * sp) + f22 * (cc * cp + d * sp));
        if (S) {
            const cd Sv[4] = {S1, S2, S3, S4};
            for (int j = 0; j < 4; ++j) {
                S[(size_t)k * 8 + 2 * j] = Sv[j].real();
                S[(size_t)k * 8 + 2 * j + 1] = Sv[j].imag();
            }
        }
        if (mu) {
            const double n1 = std::norm(S1), n2 = std::norm(S2), n3 = std::norm(S3), n4 = std::norm(S4);
            double* M = mu + (size_t)k * 16;
            M[0] = (n1 + n2 + n3 + n4) / 2;
            M[1] = (n2 - n1 + n4 - n3) / 2;
            M[2] = std::real(S2 * std::conj(S3) + S1 * std::conj(S4));
            M[3] = std::imag(S2 * std::conj(S3) - S1 * std::conj(S4));
            M[4] = (n2 - n1 + n3 - n4) / 2;
            M[5] = (n1 + n2 - n3 - n4) / 2;
            M[6] = std::real(S2 * std::conj(S3) - S1 * std::conj(S4));
            M[7] = std::imag(S2 * std::conj(S3) + S1 * std::conj(S4));
            M[8] = std::real(S2 * std::conj(S4) + S1 * std::conj(S3));
            M[9] = std::real(S2 * std::conj(S4) - S1 * std::conj(S3));
            M[10] = std::real(S1 * std::conj(S2) + S3 * std::conj(S4));
            M[11] = std::imag(S2 * std::conj(S1) + S4 * std::conj(S3));
            M[12] = std::imag(S4 * std::conj(S2) + S1 * std::conj(S3));
            M[13] = std::imag(S4 * std::conj(S2) - S1 * std::conj(S3));
            M[14] = std::imag(S1 * std::conj(S2) - S3 * std::conj(S4));
            M[15] = std::real(S1 * std::conj(S2) - S3 * std::conj(S4));
        }
    }
    return DDA_OK;
}

dda_status dda_polarization(int32_t ndir, const double* mu, double k, const double* stokes_in, double* out) {
    if (ndir <= 0 || !mu || !stokes_in || !out || !(k > 0) || !(stokes_in[0] > 0)) return DDA_ERR_INVALID_ARG;
    const double q = stokes_in[1] / stokes_in[0], u = stokes_in[2] / stokes_in[0], v = stokes_in[3] / stokes_in[0];
    const double k2 = k * k;
    for (int d = 0; d < ndir; ++d) {
        const double* M = mu + (size_t)d * 16;
        // scattered I and Q times r^2 per unit incident intensity
        const double is = (M[0] + M[1] * q + M[2] * u + M[3] * v) / k2;
        const double qs = (M[4] + M[5] * q + M[6] * u + M[7] * v) / k2;
        double* o = out + (size_t)d * 4;
        o[0] = 0.5 * (is + qs);  // polarizer parallel to the scattering plane
        o[1] = 0.5 * (is - qs);  // perpendicular to it
        o[2] = is;
        o[3] = M[0] > 0 ? std::sqrt(M[4] * M[4] + M[8] * M[8]) / M[0] : 0.0;
    }
    return DDA_OK;
}

dda_status dda_lab_frame(double beta, double theta, double phi, const double* a1in, const double* a2in, double* out) {
    if (!out) return DDA_ERR_INVALID_ARG;
    double a1[3] = {1, 0, 0}, a2[3] = {0, 1, 0};
    if (a1in) std::memcpy(a1, a1in, sizeof a1);
    if (a2in) std::memcpy(a2, a2in, sizeof a2);
    const double n1 = std::sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]);
    const double n2 = std::sqrt(a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2]);
    if (!(n1 > 0) || !(n2 > 0)) return DDA_ERR_INVALID_ARG;
    for (int i = 0; i < 3; ++i) a1[i] /= n1, a2[i] /= n2;
    const double a3[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2], a1[0] * a2[1] - a1[1] * a2[0]};
    const double cb = std::cos(beta), sb = std::sin(beta), ct = std::cos(theta), st = std::sin(theta);
    const double cp = std::cos(phi), sp = std::sin(phi);
    // coefficients of x_LF, y_LF, z_LF on (a1, a2, a3)
    const double X[3] = {ct, -st * cb, st * sb};
    const double Y[3] = {st * cp, ct * cb * cp - sb * sp, -(ct * sb * cp + cb * sp)};
    const double Z[3] = {st * sp, ct * cb * sp + sb * cp, -(ct * sb * sp - cb * cp)};
    const double* rows[3] = {X, Y, Z};
    for (int r = 0; r < 3; ++r)
        for (int i = 0; i < 3; ++i) out[3 * r + i] = rows[r][0] * a1[i] + rows[r][1] * a2[i] + rows[r][2] * a3[i];
    return DDA_OK;
}

dda_status dda_orientation_waves(double beta, double theta, double phi, const double* a1, const double* a2,
                                 const double* e01, int32_t target, dda_wave* out) {
    if (!out) return DDA_ERR_INVALID_ARG;
    double L[9];
    dda_status s = dda_lab_frame(beta, theta, phi, a1, a2, L);
    if (s < 0) return s;
    cd e1[3] = {cd(0, 0), cd(1, 0), cd(0, 0)};
    if (e01)
        for (int j = 0; j < 3; ++j) e1[j] = cd(e01[2 * j], e01[2 * j + 1]);
    const double nrm = std::sqrt(std::norm(e1[0]) + std::norm(e1[1]) + std::norm(e1[2]));
    if (!(nrm > 0)) return DDA_ERR_INVALID_ARG;
    for (auto& v : e1) v /= nrm;
    // e02 = x_LF x conj(e01) in lab components
    const cd c1[3] = {std::conj(e1[0]), std::conj(e1[1]), std::conj(e1[2])};
    const cd e2[3] = {cd(0, 0), -c1[2], c1[1]};
    const cd* es[2] = {e1, e2};
    for (int w = 0; w < 2; ++w) {
        for (int i = 0; i < 3; ++i) {
            out[w].khat[i] = L[i];
            cd v = es[w][0] * L[i] + es[w][1] * L[3 + i] + es[w][2] * L[6 + i];
            out[w].e0[2 * i] = v.real();
            out[w].e0[2 * i + 1] = v.imag();
        }
        out[w].target = target;
        out[w].pad_ = 0;
    }
    return DDA_OK;
}

dda_status dda_orientation_samples(const double* lims, const int32_t* counts, double* beta, double* theta, double* phi,
                                   double* weight) {
    if (!lims || !counts || !beta || !theta || !phi || !weight) return DDA_ERR_INVALID_ARG;
    const int nb = counts[0], nt = counts[1], np = counts[2];
    if (nb < 1 || nt < 1 || np < 1) return DDA_ERR_INVALID_ARG;
    for (int i = 0; i < nb; ++i) beta[i] = lims[0] + (i + 0.5) * (lims[1] - lims[0]) / nb;
    for (int i = 0; i < np; ++i) phi[i] = lims[4] + (i + 0.5) * (lims[5] - lims[4]) / np;
    // Theta uniform in cos(Theta): both ends and Simpson's rule for odd counts,
    // interval midpoints and equal weights for even counts
    const double u0 = std::cos(lims[2]), u1 = std::cos(lims[3]);
    std::vector<double> wt(nt);
    for (int j = 0; j < nt; ++j) {
        double u;
        if (nt == 1) {
            theta[j] = lims[2];
            wt[j] = 1;
            continue;
        }
        if (nt % 2) {
            u = u0 + j * (u1 - u0) / (nt - 1);
            wt[j] = (j == 0 || j == nt - 1) ? 1.0 : (j % 2 ? 4.0 : 2.0);
            wt[j] /= 3.0 * (nt - 1);
        } else {
            u = u0 + (j + 0.5) * (u1 - u0) / nt;
            wt[j] = 1.0 / nt;
        }
        theta[j] = std::acos(std::max(-1.0, std::min(1.0, u)));
    }
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nt; ++j)
            for (int k = 0; k < np; ++k) weight[((size_t)i * nt + j) * np + k] = wt[j] / ((double)nb * np);
    return DDA_OK;
}

dda_status dda_phi_coefficients(double beta, double theta, double phi_ref, int32_t nphi, const double* phi,
                                const double* a1, const double* a2, const double* e01, double* coeffs) {
    if (nphi < 1 || !phi || !coeffs) return DDA_ERR_INVALID_ARG;
    dda_wave ref[2], w[2];
    dda_status s = dda_orientation_waves(beta, theta, phi_ref, a1, a2, e01, 0, ref);
    if (s < 0) return s;
    for (int k = 0; k < nphi; ++k) {
        if ((s = dda_orientation_waves(beta, theta, phi[k], a1, a2, e01, 0, w)) < 0) return s;
        for (int l = 0; l < 2; ++l)
            for (int a = 0; a < 2; ++a) {
                cd v = 0;
                for (int i = 0; i < 3; ++i)
                    v += std::conj(cd(ref[a].e0[2 * i], ref[a].e0[2 * i + 1])) * cd(w[l].e0[2 * i], w[l].e0[2 * i + 1]);
                coeffs[((size_t)k * 2 + l) * 4 + 2 * a] = v.real();
                coeffs[((size_t)k * 2 + l) * 4 + 2 * a + 1] = v.imag();
            }
    }
    return DDA_OK;
}

dda_status dda_scattering_quadrature(double x, double eta, const double* L, int32_t cap, int32_t* ndir, double* n_tf,
                                     double* w) {
    if (!(x > 0) || !(eta > 0) || !L || !ndir) return DDA_ERR_INVALID_ARG;
    // theta_j at equal steps of s(theta) = theta + theta / (theta + theta0)
    const double th0 = 2 * PI / (1 + x);
    const double nr = 1 + 2 * (3 + x) / eta * (1 + 1 / (PI + th0)) / (1 + th0 / ((PI + th0) * (PI + th0)));
    const double nrc = std::min(nr, 1.0e6);
    const int nth = std::max(3, (int)std::lround(nrc));
    std::vector<double> th(nth);
    for (int j = 0; j < nth; ++j) {
        const double sj = j * PI / (nth - 1) * (1 + 1 / (PI + th0));
        th[j] = ((sj - 1 - th0) + std::sqrt((1 + th0 - sj) * (1 + th0 - sj) + 4 * th0 * sj)) / 2;
    }
    th[0] = 0;
    th[nth - 1] = PI;
    std::vector<int> nph(nth);
    long long tot = 0;
    for (int j = 0; j < nth; ++j) {
        nph[j] = (j == 0 || j == nth - 1)
                     ? 1
                     : std::max(3, (int)std::lround(4 * PI * std::sin(th[j]) / (th[j + 1] - th[j - 1])));
        tot += nph[j];
    }
    if (tot > (1LL << 30)) return DDA_ERR_INVALID_ARG;
    *ndir = (int32_t)tot;
    if (!n_tf || !w) return DDA_OK;  // size query
    if (cap < tot) return DDA_ERR_INVALID_ARG;
    long long d = 0;
    for (int j = 0; j < nth; ++j) {
        double wj;
        if (j == 0)
            wj = 2 * PI / nph[j] * (1 - (std::cos(th[0]) + std::cos(th[1])) / 2);
        else if (j == nth - 1)
            wj = 2 * PI / nph[j] * ((std::cos(th[nth - 2]) + std::cos(th[nth - 1])) / 2 + 1);
        else
            wj = PI / nph[j] * (std::cos(th[j - 1]) - std::cos(th[j + 1]));
        for (int kk = 0; kk < nph[j]; ++kk, ++d) {
            const double ph = 2 * PI * kk / nph[j];
            const double nl[3] = {std::cos(th[j]), std::sin(th[j]) * std::cos(ph), std::sin(th[j]) * std::sin(ph)};
            for (int i = 0; i < 3; ++i) n_tf[3 * d + i] = nl[0] * L[i] + nl[1] * L[3 + i] + nl[2] * L[6 + i];
            w[d] = wj;
        }
    }
    return DDA_OK;
}

dda_status dda_scattering_frame(int32_t ndir, const double* theta, const double* phi, const double* L, double* n_tf,
                                double* e_tf) {
    if (ndir <= 0 || !theta || !phi || !L || !n_tf || !e_tf) return DDA_ERR_INVALID_ARG;
    for (int d = 0; d < ndir; ++d) {
        const double ct = std::cos(theta[d]), st = std::sin(theta[d]), cp = std::cos(phi[d]), sp = std::sin(phi[d]);
        const double nl[3] = {ct, st * cp, st * sp}, tl[3] = {-st, ct * cp, ct * sp}, pl[3] = {0, -sp, cp};
        for (int i = 0; i < 3; ++i) {
            n_tf[3 * d + i] = nl[0] * L[i] + nl[1] * L[3 + i] + nl[2] * L[6 + i];
            e_tf[6 * d + i] = tl[0] * L[i] + tl[1] * L[3 + i] + tl[2] * L[6 + i];
            e_tf[6 * d + 3 + i] = pl[0] * L[i] + pl[1] * L[3 + i] + pl[2] * L[6 + i];
        }
    }
    return DDA_OK;
}

dda_status dda_set_guess_model(dda_ctx* c, dda_nn* nn) {
    if (!c) return DDA_ERR_INVALID_ARG;
    c->nn = nn;
    return DDA_OK;
}

dda_status dda_nn_record(dda_ctx* c, dda_nn* nn) {
    SCHK(check_ctx(c));
    if (!nn) return fail(c, DDA_ERR_INVALID_ARG, "nn_record: null network");
    if (!c->have_solution) return fail(c, DDA_ERR_STATE, "nn_record before a solve");
    for (auto& gp : c->groups)
        if (!gp->has_r)
            return fail(c, DDA_ERR_STATE, "nn_record needs a solve with guess PROJECT or NN");
    // sigma of every slot from the device norms of its residual field
    for (auto& gp : c->groups) {
        Group& g = *gp;
        const Target& t = *c->tg[g.tgt];
        std::vector<double> n2(g.nr);
        HCHK(c, hipMemcpy(n2.data(), g.rfn2.p, g.nr * sizeof(double), hipMemcpyDeviceToHost));
        g.hrscale.resize(g.nr);
        for (int s = 0; s < g.nr; ++s) g.hrscale[s] = (float)std::max(std::sqrt(n2[s] / (3.0 * t.N)), 1e-30);
    }
    for (int i = 0; i < c->last_nrhs; ++i) {
        Group& g = *c->groups[c->rhs_group[i]];
        Target& t = *c->tg[g.tgt];
        const int s = c->rhs_slot[i];
        hipError_t e = nn_record_one(nn, site_view(t), c->last_waves[i],
                                     reinterpret_cast<const double*>(g.hainv.data()) + (size_t)s * 2 * t.ncomp,
                                     g.x64.as<Cx<double>>() + (size_t)s * 3 * t.Npad,
                                     g.esh.as<Cx<float>>() + (size_t)s * 3 * t.Npad,
                                     g.rf.as<Cx<float>>() + (size_t)s * 3 * t.Npad, g.hrscale[s], c->stream);
        if (e == hipErrorNotSupported)
            return fail(c, DDA_ERR_UNSUPPORTED_DIMS, "nn_record: needs a cubic box with side divisible by 16");
        if (e == hipErrorInvalidValue) return fail(c, DDA_ERR_INVALID_ARG, "nn_record: all samples must share one box size");
        HCHK(c, e);
    }
    return DDA_OK;
}

dda_status dda_last_guess_ms(const dda_ctx* c, double* ms) {
    if (!c || !ms) return DDA_ERR_INVALID_ARG;
    *ms = c->ms_guess;
    return DDA_OK;
}

dda_status dda_last_timing(const dda_ctx* c, double* a, double* b, double* t) {
    if (!c) return DDA_ERR_INVALID_ARG;
    if (a) *a = c->ms_mv32;
    if (b) *b = c->ms_mv64;
    if (t) *t = c->ms_total;
    return DDA_OK;
}

}  // extern "C"

// ---- per-pass profiling and autotuning ----
namespace {
template <class T>
dda_status profile_passes(dda_ctx* c, Target& t, int nrhs, int reps, const MvShape& sh, double* ms, double* bytes) {
    hipStream_t st = c->stream;
    Group g;
    g.tgt = 0;
    g.nr = nrhs;
    const size_t ve = vec_elems(t, nrhs);
    DevMem vx, vy, ai, slab;
    HCHK(c, vx.ensure(ve * sizeof(Cx<T>)));
    HCHK(c, vy.ensure(ve * sizeof(Cx<T>)));
    HCHK(c, ai.ensure((size_t)nrhs * t.ncomp * sizeof(Cx<T>)));
    HCHK(c, slab.ensure(slab_elems(t, nrhs) * sizeof(Cx<T>)));
    HCHK(c, hipMemsetAsync(vx.p, 0, vx.n, st));
    HCHK(c, hipMemsetAsync(ai.p, 0, ai.n, st));
    const Geo geo = t.geo();
    const Tw<T> tw = t.tw<T>();
    hipEvent_t ev[4];
    for (auto& e : ev) HCHK(c, hipEventCreate(&e));
    double acc[3] = {0, 0, 0};
    for (int r = -1; r < reps; ++r) {
        HCHK(c, hipEventRecord(ev[0], st));
        for (int w = 0; w < 3; ++w) {
            HCHK(c, launch_pass<T>(w, geo, tw, t.plans, sh, nrhs, vx.as<Cx<T>>(), vy.as<Cx<T>>(), nullptr,
                                   slab.as<Cx<T>>(), t.ghat_for<T>(sh), ai.as<Cx<T>>(), nullptr, MV_AX, st));
            HCHK(c, hipEventRecord(ev[w + 1], st));
        }
        HCHK(c, hipEventSynchronize(ev[3]));
        if (r < 0) continue;  // warm-up
        for (int w = 0; w < 3; ++w) {
            float m = 0;
            HCHK(c, hipEventElapsedTime(&m, ev[w], ev[w + 1]));
            acc[w] += m;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (ms)
        for (int w = 0; w < 3; ++w) ms[w] = acc[w] / std::max(1, reps);
    if (bytes) {
        const double cb = sizeof(Cx<T>);
        const double slabb = (double)nrhs * 3 * 4 * t.n[0] * t.n[1] * t.n[2] * cb;
        const double vecb = (double)nrhs * 3 * t.N * cb;
        const double idx = (double)nrhs * 3 * t.N * 4.0;  // site coordinates read per plane pass
        const double ghb = (double)ghat_octant_elems(t.n[0], t.n[1], t.n[2]) * cb;
        bytes[0] = vecb + idx + slabb;
        bytes[1] = 2 * slabb + ghb;
        bytes[2] = slabb + 2 * vecb + idx;
    }
    return DDA_OK;
}
}  // namespace

extern "C" dda_status dda_profile_matvec(dda_ctx* c, int32_t target, int32_t nrhs, uint32_t prec, int32_t reps,
                                         double* ms, double* bytes) {
    SCHK(check_ctx(c));
    if (target < 0 || target >= (int)c->tg.size() || nrhs <= 0 || reps <= 0)
        return fail(c, DDA_ERR_INVALID_ARG, "profile_matvec: bad arguments");
    Target& t = *c->tg[target];
    SCHK(ensure_green(c, t, prec | DDA_FP64));
    if (prec == DDA_FP32) return profile_passes<float>(c, t, nrhs, reps, t.sh32, ms, bytes);
    if (prec == DDA_FP64) return profile_passes<double>(c, t, nrhs, reps, t.sh64, ms, bytes);
    return fail(c, DDA_ERR_INVALID_ARG, "profile_matvec: prec must be FP32 or FP64");
}

namespace {
// Candidate launch shapes of a target for precision T (all feasible).
template <class T>
std::vector<MvShape> shape_candidates(const Target& t) {
    std::vector<MvShape> out;
    const Geo g = t.geo();
    const MvShape base = default_shape<T>(t, 16);
    if (ct_supported(g.n1, g.n2, g.n3)) {
        for (int tx : {8, 16, 32})
            for (int zrb : {0, 1, 2, 3, 4})
                for (int pv : {0, 4, 8, 12}) {  // inverse plane pass variant, slab layout
                    MvShape c = base;
                    c.tx = tx;
                    const int av = ct_available<T>(g.n1, tx);
                    if (!(av & 2) || (pv & ~av)) continue;
                    c.ct = (av & 3) | pv;
                    c.zrb = zrb;
                    c.fused = 1;
                    if (matvec_shape_ok<T>(g, t.plans, c)) out.push_back(c);
                }
    }
    for (int tx : {4, 8, 16, 32})
        for (int fused : {1, 0}) {
            if (g.n1 % tx) continue;
            MvShape c = base;
            c.ct = 0;
            c.zrb = 0;
            c.fused = fused;
            c.tx = tx;
            const int bz = (g.n3 / rmin(t.plans[2])) * 6 * tx;
            c.nth_z = std::max(256, round64((bz + 3) / 4));
            if (matvec_shape_ok<T>(g, t.plans, c)) out.push_back(c);
        }
    return out;
}

std::string shape_key(const Target& t, int prec, int nrhs, const std::string& arch) {
    char buf[160];
    snprintf(buf, sizeof buf, "%dx%dx%d/%s/rhs%d/%s", t.n[0], t.n[1], t.n[2], prec == DDA_FP64 ? "fp64" : "fp32",
             nrhs, arch.c_str());
    return buf;
}

// Cache file: one entry per line, {"key": [fused, nth_plane, nth_z, tx, lines_tl, nth_lines, ct, zrb, ms]}.
std::vector<std::pair<std::string, std::vector<double>>> read_cache(const std::string& path) {
    std::vector<std::pair<std::string, std::vector<double>>> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t a = line.find('"'), b = line.find('"', a + 1), l = line.find('['), r = line.find(']');
        if (a == std::string::npos || b == std::string::npos || l == std::string::npos || r == std::string::npos)
            continue;
        std::vector<double> v;
        std::stringstream ss(line.substr(l + 1, r - l - 1));
        std::string tok;
        while (std::getline(ss, tok, ',')) v.push_back(std::atof(tok.c_str()));
        if (v.size() == 9) out.emplace_back(line.substr(a + 1, b - a - 1), v);
    }
    return out;
}

void write_cache(const std::string& path, const std::vector<std::pair<std::string, std::vector<double>>>& e) {
    std::ofstream f(path + ".tmp");
    f << "{\n";
    for (size_t i = 0; i < e.size(); ++i) {
        f << "  \"" << e[i].first << "\": [";
        for (size_t j = 0; j < e[i].second.size(); ++j) f << (j ? ", " : "") << e[i].second[j];
        f << "]" << (i + 1 < e.size() ? "," : "") << "\n";
    }
    f << "}\n";
    f.close();
    std::rename((path + ".tmp").c_str(), path.c_str());
}

template <class T>
dda_status tune_target(dda_ctx* c, Target& t, int nrhs, const std::string& arch,
                       std::vector<std::pair<std::string, std::vector<double>>>& cache, bool* changed) {
    const int prec = std::is_same<T, double>::value ? DDA_FP64 : DDA_FP32;
    const std::string key = shape_key(t, prec, nrhs, arch);
    MvShape& dst = std::is_same<T, double>::value ? t.sh64 : t.sh32;
    for (auto& kv : cache)
        if (kv.first == key) {
            const std::vector<double>& v = kv.second;
            MvShape s{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5], (int)v[6], (int)v[7]};
            if (matvec_shape_ok<T>(t.geo(), t.plans, s)) {
                dst = s;
                return DDA_OK;
            }
        }
    double best = 1e30;
    MvShape bs = dst;
    for (const MvShape& s : shape_candidates<T>(t)) {
        double ms[3];
        dda_status st = profile_passes<T>(c, t, nrhs, 5, s, ms, nullptr);
        if (st < 0) return st;
        const double tot = ms[0] + ms[1] + ms[2];
        if (tot < best) {
            best = tot;
            bs = s;
        }
    }
    dst = bs;
    cache.emplace_back(key, std::vector<double>{(double)bs.fused, (double)bs.nth_plane, (double)bs.nth_z, (double)bs.tx,
                                                (double)bs.lines_tl, (double)bs.nth_lines, (double)bs.ct, (double)bs.zrb,
                                                best});
    *changed = true;
    return DDA_OK;
}
}  // namespace

extern "C" dda_status dda_autotune(dda_ctx* c, int32_t nrhs_hint, const char* cache_path) {
    SCHK(check_ctx(c));
    if (c->tg.empty()) return fail(c, DDA_ERR_STATE, "autotune before set_target");
    const int nrhs = nrhs_hint > 0 ? nrhs_hint : 2;
    std::string path = cache_path ? cache_path : (std::getenv("DDA_TUNE_CACHE") ? std::getenv("DDA_TUNE_CACHE") : "");
    hipDeviceProp_t prop;
    HCHK(c, hipGetDeviceProperties(&prop, c->device));
    const std::string arch = prop.gcnArchName;
    auto cache = path.empty() ? std::vector<std::pair<std::string, std::vector<double>>>() : read_cache(path);
    bool changed = false;
    for (auto& t : c->tg) {
        SCHK(ensure_green(c, *t, DDA_FP32 | DDA_FP64));
        SCHK(tune_target<float>(c, *t, nrhs, arch, cache, &changed));
        SCHK(tune_target<double>(c, *t, nrhs, arch, cache, &changed));
    }
    if (changed && !path.empty()) write_cache(path, cache);
    c->ws_gen++;  // launch shapes are baked into captured graphs
    return DDA_OK;
}

extern "C" dda_status dda_get_shape(const dda_ctx* c, int32_t target, uint32_t prec, int32_t* out8) {
    if (!c || target < 0 || target >= (int)c->tg.size() || !out8) return DDA_ERR_INVALID_ARG;
    const MvShape& s = prec == DDA_FP64 ? c->tg[target]->sh64 : c->tg[target]->sh32;
    const int v[8] = {s.fused, s.nth_plane, s.nth_z, s.tx, s.lines_tl, s.nth_lines, s.ct, s.zrb};
    for (int i = 0; i < 8; ++i) out8[i] = v[i];
    return DDA_OK;
}

extern "C" dda_status dda_set_shape(dda_ctx* c, int32_t target, uint32_t prec, const int32_t* in8) {
    SCHK(check_ctx(c));
    if (target < 0 || target >= (int)c->tg.size() || !in8) return fail(c, DDA_ERR_INVALID_ARG, "set_shape: bad args");
    Target& t = *c->tg[target];
    MvShape s{in8[0], in8[1], in8[2], in8[3], in8[4], in8[5], in8[6], in8[7]};
    const bool ok = prec == DDA_FP64 ? matvec_shape_ok<double>(t.geo(), t.plans, s)
                                     : matvec_shape_ok<float>(t.geo(), t.plans, s);
    if (!ok) return fail(c, DDA_ERR_INVALID_ARG, "set_shape: infeasible launch shape");
    (prec == DDA_FP64 ? t.sh64 : t.sh32) = s;
    c->ws_gen++;
    return DDA_OK;
}
