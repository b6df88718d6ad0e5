// C ABI of the solver (declared in include/concord.h): argument checks,
// workspace, launch shapes, and the sequence set-up -> persistent sweeps ->
// dense output for one CONCORD-PCD solve.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/concord.h"
#include "gram.hpp"
#include "schedule.hpp"
#include "support.hpp"
#include "sweep.hpp"

namespace concord {

namespace {

constexpr size_t kAlign = 256;
constexpr int kOutWords = 8;
constexpr long long kSpinLimit = 1ll << 22;  // polls (~1 us each) before a barrier gives up

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Carves one stream-ordered allocation into the solve's buffers.  The free is
// stream-ordered too, and the call waits for it: when the entry point returns
// nothing of its own is still queued on the caller's stream (a free still in
// flight at process exit would leave the runtime's teardown to retire it).
struct Workspace {
    void *base = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    ~Workspace()
    {
        if (base) {
            (void)hipFreeAsync(base, stream);
            (void)hipStreamSynchronize(stream);
        }
    }
};

struct Carver {
    size_t off = 0;
    template <typename X>
    size_t take(size_t count)
    {
        size_t o = off;
        off = align_up(off + sizeof(X) * count);
        return o;
    }
};

struct Shape {
    int Gr, Gc, threads, w_lds, nr_max, nc_max, depth, rpt;
};

int cu_count()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return cus;
}

int max_shared_per_block()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 65536;
    return v;
}

// Launch shape for one solve of size p.  Small problems run in one
// workgroup; larger ones over a grid of Gr x Gc workgroups, one per CU (of
// the 1 / cu_share of the CUs the solve gets), with W blocks in LDS when they
// fit.  Rows of a workgroup are dealt to threads, at most two per thread.
// wide_max: the widest workgroup of the kernel's wide form (more than 512
// threads, one row per thread, W in HBM): wide_threads<T>() for a single
// solve, kJointWideThreads for the joint one (cu_share 2).
template <typename T>
int choose_shape(int p, const concord_options *o, Shape *sh, int cu_share = 1,
                 int wide_max = wide_threads<T>())
{
    const int cus = std::max(1, cu_count() / cu_share);
    int Gr = o ? o->row_groups : 0, Gc = o ? o->col_slices : 0;
    int threads = o ? o->block_threads : 0;
    int wl = o ? o->w_in_lds : 0;
    int depth = o ? o->pending_depth : 0;
    if (Gr < 0 || Gc < 0 || threads < 0 || (threads % 64) != 0 || depth < 0 || depth == 1 ||
        depth > 8)
        return CONCORD_EINVAL;
    // more than 512 threads: the wide kernel, W in HBM
    if (threads > 512 && (threads > wide_max || wl == 1))
        return CONCORD_EINVAL;
    if (Gr == 0 && Gc == 0) {
        if (p <= 96) {
            Gr = Gc = 1;
        } else {
            Gc = p < 512 ? 1 : (p < 2048 ? 2 : 8);
            Gr = std::max(1, cus / Gc);
            // Two populations sharing the CUs (the joint solve): fewer column
            // slices until a workgroup's rows fill at most half of 512
            // threads' waves, which leaves most waves of its workgroup to the
            // background rewrites (p = 5000: 32 x 4 per population instead of
            // 16 x 8; measured 350 ms against 370 ms, both at 768 threads)
            const int waves = (threads ? std::min(threads, 512) : 512) / 64;
            while (cu_share > 1 && Gc > 2 && 2 * (((p + Gr - 1) / Gr + 63) / 64) > waves) {
                Gc /= 2;
                Gr = std::max(1, cus / Gc);
            }
        }
    } else if (Gr == 0) {
        Gr = std::max(1, cus / Gc);
    } else if (Gc == 0) {
        Gc = std::max(1, cus / Gr);
    }
    if (Gc > p)
        Gc = p;
    if (Gr > p)
        Gr = p;
    sh->Gr = Gr;
    sh->Gc = Gc;
    sh->nr_max = (p + Gr - 1) / Gr;
    const bool auto_threads = (threads == 0);
    if (threads == 0)
        threads = (Gr * Gc == 1) ? 256 : 512;
    sh->threads = threads;
    sh->rpt = (sh->nr_max + threads - 1) / threads;
    if (sh->rpt > 2 || (threads > 512 && sh->rpt > 1))
        return CONCORD_ELAUNCH;
    if (sh->rpt < 1)
        sh->rpt = 1;
    int ncm = 0;
    for (int b = 0; b < Gc; ++b)
        ncm = std::max(ncm, slice_lo(b + 1, Gc, p) - slice_lo(b, Gc, p));
    sh->nc_max = ncm;
    const size_t cap = (size_t)max_shared_per_block();
    auto lds_need = [&](int d, bool w) {
        SweepParams<T> probe;
        memset(&probe, 0, sizeof(probe));
        probe.nr_max = sh->nr_max;
        probe.nc_max = sh->nc_max;
        probe.depth = d;
        probe.w_lds = w ? 1 : 0;
        return sweep_lds_bytes<T>(probe);
    };
    // W in LDS: updates are cheap, apply them at once (depth 2).  W in HBM:
    // hold up to 8 pending updates per row.
    const bool fits = lds_need(depth ? depth : 2, true) <= cap;
    if (wl == 1 && !fits)
        return CONCORD_EINVAL;
    sh->w_lds = (threads > 512 || wl == 2) ? 0 : (wl == 1 ? 1 : (fits ? 1 : 0));
    sh->depth = depth ? depth : (sh->w_lds ? 2 : 8);
    if (lds_need(sh->depth, sh->w_lds) > cap)
        return CONCORD_ELAUNCH;
    // W in HBM: the wide kernel by default when the rows leave at least half
    // of its waves to the background rewrites
    const int wt = wide_max;
    if (auto_threads && wt > 512 && !sh->w_lds && Gr * Gc > 1 &&
        sh->depth >= 4 && 2 * ((sh->nr_max + 63) / 64) <= wt / 64) {
        sh->threads = wt;
        sh->rpt = 1;
        // FP32 rows carry half the bytes, so shorter lists (more rewrites,
        // fewer gathers of pending S values per step) pay off there: depth 5
        // measured 236.5 ms against 245.5 ms at 8 (p = 5000, lambda = 0.1);
        // in FP64 depth 8 stays (5 is slower at lambda = 0.1)
        if (sizeof(T) == 4 && depth == 0 && cu_share == 1)
            sh->depth = 5;
    }
    return CONCORD_OK;
}

int map_hip(hipError_t e)
{
    if (e == hipSuccess)
        return CONCORD_OK;
    if (e == hipErrorOutOfMemory)
        return CONCORD_ENOMEM;
    if (e == hipErrorCooperativeLaunchTooLarge || e == hipErrorLaunchOutOfResources)
        return CONCORD_ELAUNCH;
    return CONCORD_EDEVICE;
}

#define CK_HIP(x)                            \
    do {                                     \
        hipError_t e_ = (x);                 \
        if (e_ != hipSuccess)                \
            return map_hip(e_);              \
    } while (0)

// Fixed device workspace of concord_fit_noalloc.  Each device the library
// runs on holds its own copy from its first use until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory: only the
// address that hipGetSymbolAddress returns for the current device is passed
// to kernels.
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[CONCORD_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(void **out)
{
    int dev = -1;
    CK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return CONCORD_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        CK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr)
            return CONCORD_EDEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CONCORD_OK;
}

// Greedy edge colouring of the support (edges i < j, in any order): edges in
// lexicographic order each take the smallest colour neither endpoint has
// used.  Writes each edge's colour (colour[e] for edge e of the list as
// given) and returns the number of colours m, padded to at least 2 (the
// sweep kernel's last colour publishes for the first); the partner table is
// built from the colours on the device.
int greedy_colouring(const int *edges, int ne, int p, std::vector<int> *colour_out)
{
    // the edges as (lo, hi) in lexicographic order: two stable counting passes,
    // by hi and then by lo (the pairs are distinct, so the order is total)
    const size_t n = (size_t)std::max(ne, 0);
    std::vector<int> lo(n), hi(n), cnt((size_t)p + 1), byhi(n), ord(n), deg((size_t)p, 0);
    for (size_t e = 0; e < n; ++e) {
        lo[e] = std::min(edges[2 * e], edges[2 * e + 1]);
        hi[e] = std::max(edges[2 * e], edges[2 * e + 1]);
        ++deg[lo[e]];
        ++deg[hi[e]];
    }
    auto pass = [&](const std::vector<int> &key, const int *in, int *out) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (size_t e = 0; e < n; ++e)
            ++cnt[(size_t)key[e] + 1];
        for (int v = 0; v < p; ++v)
            cnt[(size_t)v + 1] += cnt[v];
        for (size_t k = 0; k < n; ++k) {
            const int e = in ? in[k] : (int)k;
            out[cnt[key[e]]++] = e;
        }
    };
    pass(hi, nullptr, byhi.data());
    pass(lo, byhi.data(), ord.data());
    // an edge's colour is below deg(lo) + deg(hi) - 1, so each vertex's used
    // colours fit in W words
    const int dmax = p > 0 ? *std::max_element(deg.begin(), deg.end()) : 0;
    const size_t W = (size_t)(2 * dmax + 63) / 64 + 1;
    std::vector<uint64_t> used((size_t)p * W, 0);
    std::vector<int> &colour = *colour_out;
    colour.assign(n, 0);
    int m = 0;
    for (size_t k = 0; k < n; ++k) {
        const int e = ord[k];
        uint64_t *ui = &used[(size_t)lo[e] * W], *uj = &used[(size_t)hi[e] * W];
        size_t w = 0;
        while (~(ui[w] | uj[w]) == 0)
            ++w;
        const int c = (int)(64 * w) + __builtin_ctzll(~(ui[w] | uj[w]));
        ui[w] |= 1ull << (c % 64);
        uj[w] |= 1ull << (c % 64);
        colour[e] = c;
        m = std::max(m, c + 1);
    }
    return std::max(m, 2);
}

// ext_ws == nullptr: the workspace is allocated stream-ordered and freed
// before returning, and the call is timed with events.  Otherwise the
// workspace is carved from ext_ws (ext_cap bytes of device memory that the
// caller keeps), nothing is allocated and no events are created (the times
// in info read 0).
template <typename T>
int fit_impl(concord_input kind, const void *X, int64_t n64, int64_t p64, double lambda,
             double tol, int32_t maxit, const void *omega0, void *omega, concord_info *info,
             hipStream_t stream, const concord_options *opts, void *ext_ws = nullptr,
             size_t ext_cap = 0)
{
    const int p = (int)p64, n = (int)n64;
    Shape sh;
    int rc = choose_shape<T>(p, opts, &sh);
    if (rc)
        return rc;
    const Circle C = Circle::make(p);
    const int G = sh.Gr * sh.Gc;

    // Events: [0] call start, [1] call end, [2]/[3] around the Gram kernel,
    // [4]/[5] around the persistent sweep kernel (all on `stream`).
    hipEvent_t ev[6] = {};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int k = 0; k < 6; ++k)
                if (e[k])
                    (void)hipEventDestroy(e[k]);
        }
    } evg{ev};
    const bool own_ws = (ext_ws == nullptr);
    if (own_ws)
        for (int k = 0; k < 6; ++k)
            CK_HIP(hipEventCreate(&ev[k]));
    auto rec = [&](int k) { return ev[k] ? hipEventRecord(ev[k], stream) : hipSuccess; };

    // Workspace layout.
    Carver cv;
    const size_t pp = (size_t)p * p;
    const size_t oS = (kind == CONCORD_INPUT_Y) ? cv.take<T>(pp) : 0;
    const size_t oW = cv.take<T>(pp);
    // Active-set sweeps colour the support greedily: at most 2 Delta - 1 <
    // 2 p colours, so the sweep layout is sized for that many.
    const bool active = opts && opts->active_set;
    // a few active sweeps per phase: converging the coloured support far below
    // what the next full sweep will change wastes sweeps (measured best: 3)
    const int amax = active ? (opts->active_maxit > 0 ? opts->active_maxit : 3) : 0;
    const int Mmax = active ? std::max(C.m, 2 * p) : C.m;
    const long long ecap = active ? (long long)p * (p - 1) / 2 : 0;
    const size_t oOmp = cv.take<T>((size_t)G * C.m * sh.nr_max);
    const size_t oOmdp = cv.take<T>((size_t)G * sh.nr_max);
    // active-set sweeps keep the colouring's layout apart from Algorithm 1's,
    // which then needs only the support pairs and the diagonal refreshed
    const size_t oOmpT = cv.take<T>(active ? (size_t)G * Mmax * sh.nr_max : 1);
    const size_t oOmdpT = cv.take<T>(active ? (size_t)G * sh.nr_max : 1);
    const size_t oSd = cv.take<T>(p);
    const size_t PS = (size_t)sh.Gr * sh.nr_max;  // published slots per colour
    const size_t oPc = cv.take<T>(2 * (size_t)Mmax * PS);
    const size_t oPd = cv.take<T>(2 * PS);
    const size_t oFlags = cv.take<unsigned>(G);
    const int redsw = std::max(maxit, amax);
    const size_t oRed = cv.take<unsigned long long>(4 * (size_t)redsw);
    const size_t oOut = cv.take<int>(kOutWords);
    const size_t oAcc = cv.take<double>(4);
    const size_t oEdges = cv.take<int>(active ? 2 * (size_t)std::max(ecap, 1ll) : 1);
    const size_t oEcount = cv.take<int>(1);
    const size_t oPart = cv.take<int>(active ? (size_t)Mmax * p : 1);
    const size_t oColour = cv.take<int>(active ? (size_t)std::max(ecap, 1ll) : 1);
    Workspace ws;
    ws.stream = stream;
    ws.bytes = cv.off;
    if (own_ws) {
        hipError_t e = hipMallocAsync(&ws.base, ws.bytes, stream);
        if (e != hipSuccess) {
            ws.base = nullptr;
            return map_hip(e);
        }
    } else if (cv.off > ext_cap) {
        return CONCORD_ESCRATCH;
    }
    char *B = own_ws ? (char *)ws.base : (char *)ext_ws;
    CK_HIP(rec(0));
    T *S = (kind == CONCORD_INPUT_Y) ? (T *)(B + oS) : (T *)X;
    T *W = (T *)(B + oW);
    T *omp = (T *)(B + oOmp), *omdp = (T *)(B + oOmdp), *sd = (T *)(B + oSd);
    T *pc = (T *)(B + oPc), *pd = (T *)(B + oPd);
    unsigned *flags = (unsigned *)(B + oFlags);
    unsigned long long *red = (unsigned long long *)(B + oRed);
    int *out = (int *)(B + oOut);
    double *acc = (double *)(B + oAcc);
    unsigned long long *nnz = (unsigned long long *)(acc + 2);

    CK_HIP(launch_clear(flags, G, red, 4 * maxit, out, kOutWords, acc, 4, stream));
    if (kind == CONCORD_INPUT_Y) {
        CK_HIP(rec(2));
        CK_HIP(launch_gram<T>((const T *)X, n, p, S, stream));
        CK_HIP(rec(3));
    }
    CK_HIP(launch_check_copy<T>(S, p, W, omega0 == nullptr, sd, out + 4, stream));
    if (omega0)
        CK_HIP(launch_atb<T>((const T *)omega0, S, p, p, p, W, stream));
    CK_HIP(launch_init_omega<T>((const T *)omega0, p, sh.Gr, sh.Gc, sh.nr_max, omp, omdp, out + 4,
                                stream));
    CK_HIP(launch_init_publish<T>(W, p, sh.Gr, sh.nr_max, pc, pd, stream));

    SweepParams<T> P;
    memset(&P, 0, sizeof(P));
    P.S = S;
    P.sd = sd;
    P.W = W;
    P.omp = omp;
    P.omdp = omdp;
    P.pc = pc;
    P.pd = pd;
    P.flags = flags;
    P.red = red;
    P.out = out;
    P.p = p;
    P.Gr = sh.Gr;
    P.Gc = sh.Gc;
    P.maxit = maxit;
    P.w_lds = sh.w_lds;
    P.nr_max = sh.nr_max;
    P.nc_max = sh.nc_max;
    P.depth = sh.depth;
    P.rpt = sh.rpt;
    set_overlap(P, sh.threads, (size_t)max_shared_per_block());
    if (opts && opts->sync_rewrites)
        P.ovl = 0;
    P.lam = (T)lambda;
    P.tol = (T)tol;
    P.tol_coef = (sizeof(T) == 4) ? T(16.0 * 1.1920928955078125e-07) : T(0);  // 16 eps_f32
    P.spin_limit = kSpinLimit;
    P.tstamp = opts ? reinterpret_cast<unsigned long long *>(opts->device_timestamps) : nullptr;
    P.tstamp_steps = (opts && opts->device_timestamps) ? opts->timestamp_steps : 0;
    CK_HIP(rec(4));
    // active-set bookkeeping (host): reductions of the full sweeps, moves of
    // all launches, active sweeps
    std::vector<unsigned long long> full_red;
    int64_t a_moved = 0, a_moved_d = 0;
    int a_sweeps = 0;
    if (!active) {
        CK_HIP(launch_sweep<T>(P, sh.threads, stream));
    } else {
        int *edges = (int *)(B + oEdges), *ecount = (int *)(B + oEcount), *dpart = (int *)(B + oPart);
        int *dcolour = (int *)(B + oColour);
        T *ompT = (T *)(B + oOmpT), *omdpT = (T *)(B + oOmdpT);
        std::vector<unsigned long long> lred(4 * (size_t)redsw);
        std::vector<int> hcolour;  // colour of each support edge (host copy)
        int lout[kOutWords];
        // one launch of the sweep kernel from a clean barrier and reduction state
        auto run = [&](int mx) -> int {
            CK_HIP(launch_clear(flags, G, red, 4 * mx, out, 4, acc, 0, stream));
            P.maxit = mx;
            CK_HIP(launch_sweep<T>(P, sh.threads, stream));
            CK_HIP(hipMemcpyAsync(lout, out, sizeof(lout), hipMemcpyDeviceToHost, stream));
            CK_HIP(hipMemcpyAsync(lred.data(), red, sizeof(unsigned long long) * 4 * mx,
                                  hipMemcpyDeviceToHost, stream));
            CK_HIP(hipStreamSynchronize(stream));
            for (int t = 0; t < lout[0] && t < mx; ++t) {
                a_moved += (int64_t)lred[4 * (size_t)t + 2];
                a_moved_d += (int64_t)lred[4 * (size_t)t + 3];
            }
            return CONCORD_OK;
        };
        for (;;) {
            // a full sweep of Algorithm 1 decides convergence
            P.part = nullptr;
            P.m_tab = 0;
            int rc = run(1);
            if (rc)
                return rc;
            if (lout[0] >= 1)
                for (int w = 0; w < 4; ++w)
                    full_red.push_back(lred[w]);
            if (lout[4] || lout[2] || lout[3] || lout[1] || (int)(full_red.size() / 4) >= maxit)
                break;
            // colour the support of the current Omega
            CK_HIP(launch_finalize<T>(omp, omdp, sh.Gr, sh.Gc, sh.nr_max, W, p, (T)lambda,
                                      (T *)omega, acc, nnz, out + 4, stream));
            CK_HIP(launch_clear(nullptr, 0, nullptr, 0, ecount, 1, nullptr, 0, stream));
            CK_HIP(launch_support_edges<T>((const T *)omega, p, ecount, edges, ecap, stream));
            int ne = 0;
            CK_HIP(hipMemcpyAsync(&ne, ecount, sizeof(int), hipMemcpyDeviceToHost, stream));
            CK_HIP(hipStreamSynchronize(stream));
            std::vector<int> he(2 * (size_t)std::max(ne, 1));
            if (ne > 0) {
                CK_HIP(hipMemcpyAsync(he.data(), edges, sizeof(int) * 2 * (size_t)ne,
                                      hipMemcpyDeviceToHost, stream));
                CK_HIP(hipStreamSynchronize(stream));
            }
            const int mt = greedy_colouring(he.data(), ne, p, &hcolour);
            if (ne > 0)
                CK_HIP(hipMemcpyAsync(dcolour, hcolour.data(), sizeof(int) * (size_t)ne,
                                      hipMemcpyHostToDevice, stream));
            CK_HIP(launch_partner_table(edges, dcolour, ne, p, mt, dpart, stream));
            CK_HIP(hipStreamSynchronize(stream));
            // the sweep layout of that colouring, from the dense Omega
            CK_HIP(launch_init_omega<T>((const T *)omega, p, sh.Gr, sh.Gc, sh.nr_max, ompT, omdpT,
                                        out + 4, stream, dpart, mt));
            CK_HIP(launch_init_publish<T>(W, p, sh.Gr, sh.nr_max, pc, pd, stream, dpart, mt));
            P.part = dpart;
            P.m_tab = mt;
            P.omp = ompT;
            P.omdp = omdpT;
            rc = run(amax);
            P.omp = omp;
            P.omdp = omdp;
            if (rc)
                return rc;
            a_sweeps += lout[0];
            if (lout[4] || lout[2] || lout[3])
                break;
            // back to Algorithm 1's layout: only the coloured support pairs and
            // the diagonal moved since it was last written
            CK_HIP(launch_fill<T>((T *)omega, (long long)pp, T(0), stream));
            CK_HIP(launch_scatter_omega<T>(ompT, omdpT, dpart, mt, sh.Gr, sh.Gc, sh.nr_max, p,
                                           (T *)omega, stream));
            CK_HIP(launch_refresh_layout<T>((const T *)omega, edges, ne, p, sh.Gr, sh.Gc,
                                            sh.nr_max, omp, omdp, stream));
            CK_HIP(launch_init_publish<T>(W, p, sh.Gr, sh.nr_max, pc, pd, stream));
        }
        P.part = nullptr;
        CK_HIP(launch_clear(nullptr, 0, nullptr, 0, nullptr, 0, acc, 4, stream));
    }
    CK_HIP(rec(5));
    CK_HIP(launch_finalize<T>(omp, omdp, sh.Gr, sh.Gc, sh.nr_max, W, p, (T)lambda, (T *)omega, acc,
                              nnz, out + 4, stream));
    if (opts && opts->w_out)
        CK_HIP(hipMemcpyAsync(opts->w_out, W, sizeof(T) * pp, hipMemcpyDeviceToDevice, stream));
    CK_HIP(rec(1));

    // One readback: status words, summary accumulators and the per-sweep
    // reductions (2 * maxit words, a few KB).
    int hout[kOutWords];
    double hacc[2];
    unsigned long long hnnz = 0;
    std::vector<unsigned long long> hred(4 * (size_t)redsw);
    CK_HIP(hipMemcpyAsync(hout, out, sizeof(hout), hipMemcpyDeviceToHost, stream));
    CK_HIP(hipMemcpyAsync(hacc, acc, sizeof(hacc), hipMemcpyDeviceToHost, stream));
    CK_HIP(hipMemcpyAsync(&hnnz, nnz, sizeof(hnnz), hipMemcpyDeviceToHost, stream));
    CK_HIP(hipMemcpyAsync(hred.data(), red, sizeof(unsigned long long) * hred.size(),
                          hipMemcpyDeviceToHost, stream));
    CK_HIP(hipStreamSynchronize(stream));
    float ms = 0.f, ms_gram = 0.f, ms_sweep = 0.f;
    if (own_ws) {
        (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (kind == CONCORD_INPUT_Y)
            (void)hipEventElapsedTime(&ms_gram, ev[2], ev[3]);
        (void)hipEventElapsedTime(&ms_sweep, ev[4], ev[5]);
    }

    auto bits_to = [](unsigned long long u) -> double {
        if (sizeof(T) == 8) {
            double d;
            memcpy(&d, &u, 8);
            return d;
        }
        uint32_t w = (uint32_t)u;
        float f;
        memcpy(&f, &w, 4);
        return (double)f;
    };
    double *trace = opts ? opts->delta_trace : nullptr;
    unsigned long long last[2] = {0, 0};
    int64_t moved = 0, moved_d = 0;
    int sweeps = hout[0];
    if (!active) {
        if (trace)
            for (int t = 0; t < sweeps && t < maxit; ++t)
                trace[t] = bits_to(hred[4 * (size_t)t]);
        for (int t = 0; t < sweeps && t < maxit; ++t) {
            moved += (int64_t)hred[4 * (size_t)t + 2];
            moved_d += (int64_t)hred[4 * (size_t)t + 3];
        }
        if (sweeps > 0) {
            last[0] = hred[4 * (size_t)(sweeps - 1)];
            last[1] = hred[4 * (size_t)(sweeps - 1) + 1];
        }
    } else {
        // sweeps counts the full sweeps of Algorithm 1 (the ones that decide
        // convergence); moves are those of every sweep
        sweeps = (int)(full_red.size() / 4);
        if (trace)
            for (int t = 0; t < sweeps && t < maxit; ++t)
                trace[t] = bits_to(full_red[4 * (size_t)t]);
        moved = a_moved;
        moved_d = a_moved_d;
        if (sweeps > 0) {
            last[0] = full_red[4 * (size_t)(sweeps - 1)];
            last[1] = full_red[4 * (size_t)(sweeps - 1) + 1];
        }
    }
    const double delta = bits_to(last[0]);
    const double gmax = bits_to(last[1]);
    const double tol_eff = std::max(tol, (double)P.tol_coef * gmax);

    int status;
    if (hout[4] & kErrNotPD)
        status = CONCORD_ENOTPD;
    else if (hout[4] & kErrNonFinite)
        status = CONCORD_ENONFINITE;
    else if (hout[2] || hout[3])
        status = CONCORD_EDEVICE;
    else
        status = hout[1] ? CONCORD_OK : CONCORD_NOT_CONVERGED;
    if (info) {
        info->sweeps = sweeps;
        info->status = status;
        info->delta = delta;
        info->tol_eff = tol_eff;
        info->nnz_upper = (int64_t)hnnz;
        info->objective = hacc[0];
        info->elapsed_ms = ms;
        info->gram_ms = ms_gram;
        info->sweep_ms = ms_sweep;
        info->moved_pairs = moved;
        info->moved_diag = moved_d;
        info->row_groups = sh.Gr;
        info->col_slices = sh.Gc;
        info->w_in_lds = sh.w_lds;
        info->block_threads = sh.threads;
        info->pending_depth = sh.depth;
        info->active_sweeps = a_sweeps;
    }
    return status;
}

// ---------------------------------------------------------------- backward

// Implicit gradient at Omega-hat: set up the adjoint system (v = 0, U = V S =
// 0, right-hand side from grad_omega), solve it with the sweep kernel in its
// adjoint mode, then dL/dS = -(Omega V + V Omega)/2 (Omega V by the matrix-core
// product) and dL/dlam = -sum_{i<j} v_ij sign(omega_ij).
template <typename T>
int backward_impl(const void *Sv, const void *omv, int64_t p64, const void *Cv, void *gSv,
                  double *grad_lambda, double tol, int32_t maxit, concord_info *info,
                  hipStream_t stream, const concord_options *opts)
{
    const int p = (int)p64;
    Shape sh;
    int rc = choose_shape<T>(p, opts, &sh);
    if (rc)
        return rc;
    const Circle C = Circle::make(p);
    const int G = sh.Gr * sh.Gc;
    hipEvent_t ev[4] = {};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int k = 0; k < 4; ++k)
                if (e[k])
                    (void)hipEventDestroy(e[k]);
        }
    } evg{ev};
    for (int k = 0; k < 4; ++k)
        CK_HIP(hipEventCreate(&ev[k]));
    CK_HIP(hipEventRecord(ev[0], stream));

    Carver cv;
    const size_t pp = (size_t)p * p;
    const size_t oW = cv.take<T>(pp);
    const size_t oVp = cv.take<T>((size_t)G * C.m * sh.nr_max);
    const size_t oVdp = cv.take<T>((size_t)G * sh.nr_max);
    const size_t oAg = cv.take<T>((size_t)G * C.m * sh.nr_max);
    const size_t oAgd = cv.take<T>((size_t)G * sh.nr_max);
    const size_t oAhd = cv.take<T>((size_t)G * sh.nr_max);
    const size_t oSd = cv.take<T>(p);
    const size_t PS = (size_t)sh.Gr * sh.nr_max;
    const size_t oPc = cv.take<T>(2 * (size_t)C.m * PS);
    const size_t oPd = cv.take<T>(2 * PS);
    const size_t oFlags = cv.take<unsigned>(G);
    const size_t oRed = cv.take<unsigned long long>(4 * (size_t)maxit);
    const size_t oOut = cv.take<int>(kOutWords);
    const size_t oAcc = cv.take<double>(4);
    const size_t oV = cv.take<T>(pp);
    const size_t oM = cv.take<T>(pp);
    Workspace ws;
    ws.stream = stream;
    ws.bytes = cv.off;
    {
        hipError_t e = hipMallocAsync(&ws.base, ws.bytes, stream);
        if (e != hipSuccess) {
            ws.base = nullptr;
            return map_hip(e);
        }
    }
    char *B = (char *)ws.base;
    const T *S = (const T *)Sv, *om = (const T *)omv, *Cg = (const T *)Cv;
    T *W = (T *)(B + oW), *vp = (T *)(B + oVp), *vdp = (T *)(B + oVdp);
    T *adj_g = (T *)(B + oAg), *adj_gd = (T *)(B + oAgd), *adj_hd = (T *)(B + oAhd);
    T *sd = (T *)(B + oSd), *pc = (T *)(B + oPc), *pd = (T *)(B + oPd);
    T *V = (T *)(B + oV), *M = (T *)(B + oM);
    unsigned *flags = (unsigned *)(B + oFlags);
    unsigned long long *red = (unsigned long long *)(B + oRed);
    int *out = (int *)(B + oOut);
    double *acc = (double *)(B + oAcc);

    CK_HIP(launch_clear(flags, G, red, 4 * maxit, out, kOutWords, acc, 4, stream));
    CK_HIP(launch_check_copy<T>(S, p, W, false, sd, out + 4, stream));
    CK_HIP(launch_fill<T>(W, (long long)pp, T(0), stream));
    CK_HIP(launch_init_adjoint<T>(om, Cg, sd, p, sh.Gr, sh.Gc, sh.nr_max, vp, vdp, adj_g, adj_gd,
                                  adj_hd, out + 4, stream));
    CK_HIP(launch_init_publish<T>(W, p, sh.Gr, sh.nr_max, pc, pd, stream));

    SweepParams<T> P;
    memset(&P, 0, sizeof(P));
    P.S = S;
    P.sd = sd;
    P.W = W;
    P.omp = vp;
    P.omdp = vdp;
    P.pc = pc;
    P.pd = pd;
    P.flags = flags;
    P.red = red;
    P.out = out;
    P.p = p;
    P.Gr = sh.Gr;
    P.Gc = sh.Gc;
    P.maxit = maxit;
    P.w_lds = sh.w_lds;
    P.nr_max = sh.nr_max;
    P.nc_max = sh.nc_max;
    P.depth = sh.depth;
    P.rpt = sh.rpt;
    set_overlap(P, sh.threads, (size_t)max_shared_per_block());
    if (opts && opts->sync_rewrites)
        P.ovl = 0;
    P.tol = (T)tol;
    P.tol_coef = (sizeof(T) == 4) ? T(16.0 * 1.1920928955078125e-07) : T(0);
    P.spin_limit = kSpinLimit;
    P.adj_g = adj_g;
    P.adj_gd = adj_gd;
    P.adj_hd = adj_hd;
    CK_HIP(hipEventRecord(ev[1], stream));
    CK_HIP(launch_sweep<T>(P, sh.threads, stream));
    CK_HIP(hipEventRecord(ev[2], stream));
    CK_HIP(launch_gather<T>(vp, vdp, sh.Gr, sh.Gc, sh.nr_max, p, V, stream));
    CK_HIP(launch_atb<T>(om, V, p, p, p, M, stream));
    CK_HIP(launch_adjoint_output<T>(M, V, om, p, (T *)gSv, acc, out + 4, stream));
    CK_HIP(hipEventRecord(ev[3], stream));

    int hout[kOutWords];
    double hacc = 0.0;
    std::vector<unsigned long long> hred(4 * (size_t)maxit);
    CK_HIP(hipMemcpyAsync(hout, out, sizeof(hout), hipMemcpyDeviceToHost, stream));
    CK_HIP(hipMemcpyAsync(&hacc, acc, sizeof(double), hipMemcpyDeviceToHost, stream));
    CK_HIP(hipMemcpyAsync(hred.data(), red, sizeof(unsigned long long) * hred.size(),
                          hipMemcpyDeviceToHost, stream));
    CK_HIP(hipStreamSynchronize(stream));
    float ms = 0.f, ms_sweep = 0.f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[3]);
    (void)hipEventElapsedTime(&ms_sweep, ev[1], ev[2]);
    const int sweeps = hout[0];
    auto bits_to = [](unsigned long long u) -> double {
        if (sizeof(T) == 8) {
            double d;
            memcpy(&d, &u, 8);
            return d;
        }
        uint32_t w = (uint32_t)u;
        float f;
        memcpy(&f, &w, 4);
        return (double)f;
    };
    int status;
    if (hout[4] & kErrNotPD)
        status = CONCORD_ENOTPD;
    else if (hout[4] & kErrNonFinite)
        status = CONCORD_ENONFINITE;
    else if (hout[2] || hout[3])
        status = CONCORD_EDEVICE;
    else
        status = hout[1] ? CONCORD_OK : CONCORD_NOT_CONVERGED;
    if (grad_lambda)
        *grad_lambda = hacc;
    if (info) {
        memset(info, 0, sizeof(*info));
        info->sweeps = sweeps;
        info->status = status;
        if (sweeps > 0) {
            info->delta = bits_to(hred[4 * (size_t)(sweeps - 1)]);
            info->tol_eff = std::max(tol, (double)P.tol_coef * bits_to(hred[4 * (size_t)(sweeps - 1) + 1]));
        } else {
            info->tol_eff = tol;
        }
        int64_t mv = 0, mvd = 0;
        for (int t = 0; t < sweeps && t < maxit; ++t) {
            mv += (int64_t)hred[4 * (size_t)t + 2];
            mvd += (int64_t)hred[4 * (size_t)t + 3];
        }
        info->elapsed_ms = ms;
        info->sweep_ms = ms_sweep;
        info->moved_pairs = mv;
        info->moved_diag = mvd;
        info->row_groups = sh.Gr;
        info->col_slices = sh.Gc;
        info->w_in_lds = sh.w_lds;
        info->block_threads = sh.threads;
        info->pending_depth = sh.depth;
    }
    return status;
}

// ---------------------------------------------------------------- batched

// Status of a batch: the first negative code met, else NOT_CONVERGED if any
// solve stopped at maxit, else OK.
int merge_status(int acc, int s)
{
    if (acc < 0)
        return acc;
    if (s < 0)
        return s;
    return (s == CONCORD_NOT_CONVERGED || acc == CONCORD_NOT_CONVERGED) ? CONCORD_NOT_CONVERGED
                                                                         : CONCORD_OK;
}

// Workgroups for each problem of a batch sharing `total` workgroups.  Each
// problem needs ceil(p / (2 * threads)) workgroups (two rows per thread at
// most) and keeps at least 8 rows per workgroup.  The rest are dealt one at a
// time to the problem with the largest work per workgroup, work ~ p^1.55:
// along a descending lambda path with n ~ p / 2 the bytes a solve moves grow
// like that (smaller problems need more sweeps), which is what the measured
// per-problem device times of such batches follow.  Returns false when the
// minimum does not fit.
bool plan_workgroups(const std::vector<int> &ps, int total, int max_rows, std::vector<int> *G)
{
    const int B = (int)ps.size();
    G->assign(B, 1);
    long long used = 0;
    std::vector<double> w(B);
    for (int b = 0; b < B; ++b) {
        (*G)[b] = std::max(1, (ps[b] + max_rows - 1) / max_rows);
        used += (*G)[b];
        w[b] = pow((double)ps[b], 1.55);
    }
    if (used > total)
        return false;
    for (long long left = total - used; left > 0; --left) {
        int best = -1;
        double bc = -1.0;
        for (int b = 0; b < B; ++b) {
            if (((*G)[b] + 1) * 8 > ps[b])  // keep >= 8 rows per workgroup
                continue;
            const double c = w[b] / (*G)[b];
            if (c > bc) {
                bc = c;
                best = b;
            }
        }
        if (best < 0)
            break;
        ++(*G)[best];
    }
    return true;
}

template <typename T>
int batched_chunk(int B0, int B1, concord_input kind, const void *const *X, const int64_t *n,
                  const int64_t *pv, int L, const double *lambdas, double tol, int maxit,
                  void *const *omega, concord_info *info, hipStream_t stream,
                  const std::vector<int> &Gb, const std::vector<int> &Cb, int threads, int depth,
                  int cpl, bool sync_rw)
{
    const int NB = B1 - B0;
    hipEvent_t ev[4] = {};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int k = 0; k < 4; ++k)
                if (e[k])
                    (void)hipEventDestroy(e[k]);
        }
    } evg{ev};
    for (int k = 0; k < 4; ++k)
        CK_HIP(hipEventCreate(&ev[k]));

    // Per-problem shapes and workspace offsets.
    // Problem q: G = Gr x Gc workgroups (row groups x column slices).
    struct Prob {
        int p, G, Gr, Gc, nr, nc, m, ovl;
        size_t oS, oW, oOmp, oOmdp, oSd, oPc, oPd, oFlags, oRed, oOut, oRec, oLam, oOm;
    };
    std::vector<Prob> pr(NB);
    Carver cv;
    int Gtot = 0;
    size_t lds = 0;
    for (int q = 0; q < NB; ++q) {
        const int b = B0 + q;
        Prob &P = pr[q];
        P.p = (int)pv[b];
        P.G = Gb[b];
        P.Gc = Cb[b];
        P.Gr = P.G / P.Gc;
        P.nr = (P.p + P.Gr - 1) / P.Gr;
        P.nc = 0;
        for (int c = 0; c < P.Gc; ++c)
            P.nc = std::max(P.nc, slice_lo(c + 1, P.Gc, P.p) - slice_lo(c, P.Gc, P.p));
        P.m = Circle::make(P.p).m;
        const size_t pp = (size_t)P.p * P.p;
        P.oS = (kind == CONCORD_INPUT_Y) ? cv.take<T>(pp) : 0;
        P.oW = cv.take<T>(pp);
        P.oOmp = cv.take<T>((size_t)P.G * P.m * P.nr);
        P.oOmdp = cv.take<T>((size_t)P.G * P.nr);
        P.oSd = cv.take<T>(P.p);
        const size_t PS = (size_t)P.Gr * P.nr;
        P.oPc = cv.take<T>(2 * (size_t)P.m * PS);
        P.oPd = cv.take<T>(2 * PS);
        P.oFlags = cv.take<unsigned>(P.G);
        P.oRed = cv.take<unsigned long long>(4 * (size_t)L * maxit);
        P.oOut = cv.take<int>(kOutWords);
        P.oRec = cv.take<PathRec>(L);
        P.oLam = cv.take<double>(L);
        P.oOm = cv.take<T *>(L);
        SweepParams<T> probe;
        memset(&probe, 0, sizeof(probe));
        probe.nr_max = P.nr;
        probe.nc_max = P.nc;
        probe.depth = depth;
        set_overlap(probe, threads, (size_t)max_shared_per_block());
        if (sync_rw)
            probe.ovl = 0;
        P.ovl = probe.ovl;
        lds = std::max(lds, sweep_lds_bytes<T>(probe));
        Gtot += P.G;
    }
    if (lds > (size_t)max_shared_per_block())
        return CONCORD_ELAUNCH;
    const size_t oDesc = cv.take<SweepParams<T>>(NB);
    const size_t oMap = cv.take<int>(Gtot);
    Workspace ws;
    ws.stream = stream;
    ws.bytes = cv.off;
    {
        hipError_t e = hipMallocAsync(&ws.base, ws.bytes, stream);
        if (e != hipSuccess) {
            ws.base = nullptr;
            return map_hip(e);
        }
    }
    char *base = (char *)ws.base;

    // Descriptors, the workgroup -> problem map, lambda paths and output
    // pointer tables (host copies live until the final synchronisation).
    std::vector<SweepParams<T>> desc(NB);
    std::vector<int> wmap(Gtot);
    std::vector<double> hl((size_t)NB * L);
    std::vector<T *> hom((size_t)NB * L);
    CK_HIP(hipEventRecord(ev[0], stream));
    int g0 = 0;
    for (int q = 0; q < NB; ++q) {
        const int b = B0 + q;
        const Prob &P = pr[q];
        T *S = (kind == CONCORD_INPUT_Y) ? (T *)(base + P.oS) : (T *)X[b];
        T *W = (T *)(base + P.oW);
        T *omp = (T *)(base + P.oOmp), *omdp = (T *)(base + P.oOmdp), *sd = (T *)(base + P.oSd);
        T *pc = (T *)(base + P.oPc), *pd = (T *)(base + P.oPd);
        int *out = (int *)(base + P.oOut);
        CK_HIP(launch_clear((unsigned *)(base + P.oFlags), P.G,
                            (unsigned long long *)(base + P.oRed), 4 * L * maxit, out, kOutWords,
                            (double *)(base + P.oRec), (int)(sizeof(PathRec) / 8) * L, stream));
        static_assert(sizeof(PathRec) % 8 == 0, "PathRec is cleared as 8-byte words");
        if (kind == CONCORD_INPUT_Y)
            CK_HIP(launch_gram<T>((const T *)X[b], (int)n[b], P.p, S, stream));
        CK_HIP(launch_check_copy<T>(S, P.p, W, true, sd, out + 4, stream));
        CK_HIP(launch_init_omega<T>(nullptr, P.p, P.Gr, P.Gc, P.nr, omp, omdp, out + 4, stream));
        CK_HIP(launch_init_publish<T>(W, P.p, P.Gr, P.nr, pc, pd, stream));
        for (int l = 0; l < L; ++l) {
            hl[(size_t)q * L + l] = lambdas[(size_t)b * L + l];
            hom[(size_t)q * L + l] = (T *)omega[(size_t)b * L + l];
        }
        SweepParams<T> &D = desc[q];
        memset(&D, 0, sizeof(D));
        D.S = S;
        D.sd = sd;
        D.W = W;
        D.omp = omp;
        D.omdp = omdp;
        D.pc = pc;
        D.pd = pd;
        D.flags = (unsigned *)(base + P.oFlags);
        D.red = (unsigned long long *)(base + P.oRed);
        D.out = out;
        D.p = P.p;
        D.Gr = P.Gr;
        D.Gc = P.Gc;
        D.maxit = maxit;
        D.w_lds = 0;
        D.nr_max = P.nr;
        D.nc_max = P.nc;
        D.depth = depth;
        D.rpt = (threads > 512) ? 1 : 2;
        D.ovl = P.ovl;
        D.lam = (T)hl[(size_t)q * L];
        D.tol = (T)tol;
        D.tol_coef = (sizeof(T) == 4) ? T(16.0 * 1.1920928955078125e-07) : T(0);
        D.spin_limit = kSpinLimit;
        D.L = L;
        D.lams = (const double *)(base + P.oLam);
        D.omega_out = (T *const *)(base + P.oOm);
        D.rec = (PathRec *)(base + P.oRec);
        D.g0 = g0;
        for (int g = 0; g < P.G; ++g)
            wmap[g0 + g] = q;
        g0 += P.G;
        CK_HIP(hipMemcpyAsync(base + P.oLam, &hl[(size_t)q * L], sizeof(double) * L,
                              hipMemcpyHostToDevice, stream));
        CK_HIP(hipMemcpyAsync(base + P.oOm, &hom[(size_t)q * L], sizeof(T *) * L,
                              hipMemcpyHostToDevice, stream));
    }
    CK_HIP(hipMemcpyAsync(base + oDesc, desc.data(), sizeof(SweepParams<T>) * NB,
                          hipMemcpyHostToDevice, stream));
    CK_HIP(hipMemcpyAsync(base + oMap, wmap.data(), sizeof(int) * Gtot, hipMemcpyHostToDevice,
                          stream));
    CK_HIP(hipEventRecord(ev[1], stream));
    bool any_bg = false;
    for (int q = 0; q < NB; ++q)
        any_bg = any_bg || pr[q].ovl;
    if (threads > 512)
        CK_HIP(launch_sweep_batched_wide<T>((const SweepParams<T> *)(base + oDesc),
                                            (const int *)(base + oMap), Gtot, lds, threads, cpl,
                                            any_bg, stream));
    else
        CK_HIP(launch_sweep_batched<T>((const SweepParams<T> *)(base + oDesc),
                                       (const int *)(base + oMap), Gtot, lds, threads, cpl,
                                       any_bg, stream));
    CK_HIP(hipEventRecord(ev[2], stream));

    // Readback: status words, per-sweep reductions and per-lambda records.
    std::vector<int> hout((size_t)NB * kOutWords);
    std::vector<unsigned long long> hred((size_t)NB * 4 * L * maxit);
    std::vector<PathRec> hrec((size_t)NB * L);
    for (int q = 0; q < NB; ++q) {
        const Prob &P = pr[q];
        CK_HIP(hipMemcpyAsync(&hout[(size_t)q * kOutWords], base + P.oOut, sizeof(int) * kOutWords,
                              hipMemcpyDeviceToHost, stream));
        CK_HIP(hipMemcpyAsync(&hred[(size_t)q * 4 * L * maxit], base + P.oRed,
                              sizeof(unsigned long long) * 4 * L * maxit, hipMemcpyDeviceToHost,
                              stream));
        CK_HIP(hipMemcpyAsync(&hrec[(size_t)q * L], base + P.oRec, sizeof(PathRec) * L,
                              hipMemcpyDeviceToHost, stream));
    }
    CK_HIP(hipEventRecord(ev[3], stream));
    CK_HIP(hipStreamSynchronize(stream));
    float ms = 0.f, ms_setup = 0.f, ms_sweep = 0.f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[3]);
    (void)hipEventElapsedTime(&ms_setup, ev[0], ev[1]);
    (void)hipEventElapsedTime(&ms_sweep, ev[1], ev[2]);

    auto bits_to = [](unsigned long long u) -> double {
        if (sizeof(T) == 8) {
            double d;
            memcpy(&d, &u, 8);
            return d;
        }
        uint32_t w = (uint32_t)u;
        float f;
        memcpy(&f, &w, 4);
        return (double)f;
    };
    int worst = CONCORD_OK;
    for (int q = 0; q < NB; ++q) {
        const int b = B0 + q;
        const int *ho = &hout[(size_t)q * kOutWords];
        const unsigned long long *hr = &hred[(size_t)q * 4 * L * maxit];
        int pstat = CONCORD_OK;
        if (ho[4] & kErrNotPD)
            pstat = CONCORD_ENOTPD;
        else if (ho[4] & kErrNonFinite)
            pstat = CONCORD_ENONFINITE;
        else if (ho[2] || ho[3])
            pstat = CONCORD_EDEVICE;
        int t0 = 0;
        for (int l = 0; l < L; ++l) {
            const PathRec &rc = hrec[(size_t)q * L + l];
            int status = pstat;
            int t1 = rc.t_end;
            if (status == CONCORD_OK && t1 <= t0)
                status = CONCORD_EDEVICE;  // the path stopped before this lambda
            if (status == CONCORD_OK)
                status = rc.converged ? CONCORD_OK : CONCORD_NOT_CONVERGED;
            if (t1 < t0)
                t1 = t0;
            concord_info *I = info ? &info[(size_t)b * L + l] : nullptr;
            if (I) {
                memset(I, 0, sizeof(*I));
                I->sweeps = t1 - t0;
                I->status = status;
                if (t1 > t0) {
                    I->delta = bits_to(hr[4 * (size_t)(t1 - 1)]);
                    const double gmax = bits_to(hr[4 * (size_t)(t1 - 1) + 1]);
                    I->tol_eff = std::max(tol, (sizeof(T) == 4 ? 16.0 * 1.1920928955078125e-07 : 0.0) * gmax);
                } else {
                    I->tol_eff = tol;
                }
                int64_t mv = 0, mvd = 0;
                for (int t = t0; t < t1; ++t) {
                    mv += (int64_t)hr[4 * (size_t)t + 2];
                    mvd += (int64_t)hr[4 * (size_t)t + 3];
                }
                I->nnz_upper = (int64_t)rc.nnz_upper;
                I->objective = rc.objective;
                I->elapsed_ms = ms;
                I->gram_ms = ms_setup;
                // this lambda's own device time (100 MHz clock); the launch's
                // sweep time when the path stopped before it
                I->sweep_ms = (rc.clock_end > rc.clock_start)
                                  ? (double)(rc.clock_end - rc.clock_start) * 1e-5
                                  : (double)ms_sweep;
                I->moved_pairs = mv;
                I->moved_diag = mvd;
                I->row_groups = pr[q].Gr;
                I->col_slices = pr[q].Gc;
                I->w_in_lds = 0;
                I->block_threads = threads;
                I->pending_depth = depth;
            }
            worst = merge_status(worst, status);
            t0 = t1;
        }
    }
    return worst;
}

template <typename T>
int batched_impl(int B, concord_input kind, const void *const *X, const int64_t *n,
                 const int64_t *pv, int L, const double *lambdas, double tol, int maxit,
                 void *const *omega, concord_info *info, hipStream_t stream,
                 const concord_batch_options *o)
{
    const int cus = std::max(1, cu_count());
    int total = (o && o->workgroups > 0) ? o->workgroups : cus;
    // default width: wide workgroups in FP32 (they hold as many rows as 512
    // threads with two rows each, and more problems rewrite in the
    // background); 512 threads in FP64, whose wide form holds fewer rows
    int threads = (o && o->block_threads > 0) ? o->block_threads
                                              : (sizeof(T) == 4 ? wide_threads<T>() : 512);
    int depth = (o && o->pending_depth > 0) ? o->pending_depth : 8;
    const int cpl = (o && o->cols_per_lane > 0) ? o->cols_per_lane : 4;
    if (o && (o->workgroups < 0 || o->block_threads < 0 || o->pending_depth < 0 ||
              o->cols_per_lane < 0))
        return CONCORD_EINVAL;
    // co-residency of the persistent launch: one workgroup of up to 512
    // threads (or a wide one, up to wide_threads<T>(), one row per thread)
    // per CU, or two of at most 256 threads
    const int per_cu = (threads <= 256) ? 2 : 1;
    if (total > per_cu * cus || threads % 64 != 0 || threads > wide_threads<T>() || depth < 2 ||
        depth > 8 || (cpl != 2 && cpl != 4))
        return CONCORD_EINVAL;
    // rows of W a workgroup can hold: two per thread, one in a wide workgroup
    const int max_rows = (threads > 512 ? 1 : 2) * threads;
    // Problems go in order into launches of at most `total` workgroups.
    std::vector<int> minG(B);
    for (int b = 0; b < B; ++b)
        minG[b] = std::max(1, (int)((pv[b] + max_rows - 1) / max_rows));
    const int32_t *fixed = o ? o->problem_workgroups : nullptr;
    if (fixed) {
        long long sum = 0;
        for (int b = 0; b < B; ++b) {
            if (fixed[b] < minG[b] || fixed[b] > pv[b])
                return CONCORD_EINVAL;
            sum += fixed[b];
        }
        if (sum > total)
            return CONCORD_EINVAL;
    }
    const int32_t *slices = o ? o->problem_col_slices : nullptr;
    std::vector<int> Cb(B, 1);
    if (slices) {
        if (!fixed)
            return CONCORD_EINVAL;
        for (int b = 0; b < B; ++b) {
            const int c = slices[b];
            if (c < 1 || c > pv[b] || fixed[b] % c != 0)
                return CONCORD_EINVAL;
            const long long gr = fixed[b] / c;
            if ((pv[b] + gr - 1) / gr > max_rows)
                return CONCORD_EINVAL;
            Cb[b] = c;
        }
    }
    std::vector<int> Gb(B, 1);
    int worst = CONCORD_OK;
    for (int b0 = 0; b0 < B;) {
        int b1 = b0;
        long long used = 0;
        while (b1 < B && used + minG[b1] <= total)
            used += minG[b1++];
        if (b1 == b0)
            return CONCORD_ELAUNCH;
        std::vector<int> ps(pv + b0, pv + b1), G;
        if (fixed)
            G.assign(fixed + b0, fixed + b1);
        else if (!plan_workgroups(ps, total, max_rows, &G))
            return CONCORD_ELAUNCH;
        for (int b = b0; b < b1; ++b)
            Gb[b] = G[b - b0];
        const int rc = batched_chunk<T>(b0, b1, kind, X, n, pv, L, lambdas, tol, maxit, omega,
                                        info, stream, Gb, Cb, threads, depth, cpl,
                                        o && o->sync_rewrites);
        worst = merge_status(worst, rc);
        if (rc == CONCORD_ENOMEM || rc == CONCORD_EDEVICE || rc == CONCORD_ELAUNCH)
            return rc;
        b0 = b1;
    }
    return worst;
}

// ---------------------------------------------------------------- joint

// Joint estimation of two precision matrices (Section 6): per population the
// set-up of a single solve plus a copy of the other population's starting
// omega in the layout of this population's workgroups, one persistent launch
// of both, then each population's dense output and the fused term.
template <typename T>
int joint_impl(concord_input kind, const void *const X[2], const int64_t n[2], int64_t p64,
               double lam1, double lam2, double tol, int32_t maxit, const void *const omega0[2],
               void *const omega[2], concord_joint_info *info, hipStream_t stream,
               const concord_options *opts)
{
    const int p = (int)p64;
    if (opts && (opts->active_set || opts->w_out || opts->device_timestamps))
        return CONCORD_EINVAL;
    Shape sh;
    int rc = choose_shape<T>(p, opts, &sh, 2, kJointWideThreads);
    if (rc)
        return rc;
    const Circle C = Circle::make(p);
    const int G = sh.Gr * sh.Gc;

    hipEvent_t ev[6] = {};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int k = 0; k < 6; ++k)
                if (e[k])
                    (void)hipEventDestroy(e[k]);
        }
    } evg{ev};
    for (int k = 0; k < 6; ++k)
        CK_HIP(hipEventCreate(&ev[k]));
    CK_HIP(hipEventRecord(ev[0], stream));

    Carver cv;
    const size_t pp = (size_t)p * p;
    const size_t PS = (size_t)sh.Gr * sh.nr_max;
    size_t oS[2], oW[2], oOmp[2], oOmdp[2], oSd[2], oPc[2], oPd[2], oOx[2], oOdx[2];
    for (int m = 0; m < 2; ++m) {
        oS[m] = (kind == CONCORD_INPUT_Y) ? cv.take<T>(pp) : 0;
        oW[m] = cv.take<T>(pp);
        oOmp[m] = cv.take<T>((size_t)G * C.m * sh.nr_max);
        oOmdp[m] = cv.take<T>((size_t)G * sh.nr_max);
        oOx[m] = cv.take<T>((size_t)G * C.m * sh.nr_max);
        oOdx[m] = cv.take<T>((size_t)G * sh.nr_max);
        oSd[m] = cv.take<T>(p);
        oPc[m] = cv.take<T>(2 * (size_t)C.m * PS);
        oPd[m] = cv.take<T>(2 * PS);
    }
    const size_t oFlags = cv.take<unsigned>(2 * (size_t)G);
    const size_t oRed = cv.take<unsigned long long>(4 * (size_t)maxit);
    const size_t oOut = cv.take<int>(kOutWords);
    const size_t oAcc = cv.take<double>(8);  // [0..2] objectives and fused term, [4..6] counts
    Workspace ws;
    ws.stream = stream;
    ws.bytes = cv.off;
    {
        hipError_t e = hipMallocAsync(&ws.base, ws.bytes, stream);
        if (e != hipSuccess) {
            ws.base = nullptr;
            return map_hip(e);
        }
    }
    char *B = (char *)ws.base;
    T *S[2], *W[2], *omp[2], *omdp[2], *ox[2], *odx[2], *sd[2], *pc[2], *pd[2];
    for (int m = 0; m < 2; ++m) {
        S[m] = (kind == CONCORD_INPUT_Y) ? (T *)(B + oS[m]) : (T *)X[m];
        W[m] = (T *)(B + oW[m]);
        omp[m] = (T *)(B + oOmp[m]);
        omdp[m] = (T *)(B + oOmdp[m]);
        ox[m] = (T *)(B + oOx[m]);
        odx[m] = (T *)(B + oOdx[m]);
        sd[m] = (T *)(B + oSd[m]);
        pc[m] = (T *)(B + oPc[m]);
        pd[m] = (T *)(B + oPd[m]);
    }
    unsigned *flags = (unsigned *)(B + oFlags);
    unsigned long long *red = (unsigned long long *)(B + oRed);
    int *out = (int *)(B + oOut);
    double *acc = (double *)(B + oAcc);
    unsigned long long *cnt = (unsigned long long *)(acc + 4);

    CK_HIP(launch_clear(flags, 2 * G, red, 4 * maxit, out, kOutWords, acc, 8, stream));
    if (kind == CONCORD_INPUT_Y) {
        CK_HIP(hipEventRecord(ev[2], stream));
        for (int m = 0; m < 2; ++m)
            CK_HIP(launch_gram<T>((const T *)X[m], (int)n[m], p, S[m], stream));
        CK_HIP(hipEventRecord(ev[3], stream));
    }
    for (int m = 0; m < 2; ++m) {
        CK_HIP(launch_check_copy<T>(S[m], p, W[m], omega0[m] == nullptr, sd[m], out + 4, stream));
        if (omega0[m])
            CK_HIP(launch_atb<T>((const T *)omega0[m], S[m], p, p, p, W[m], stream));
        CK_HIP(launch_init_omega<T>((const T *)omega0[m], p, sh.Gr, sh.Gc, sh.nr_max, omp[m],
                                    omdp[m], out + 4, stream));
        CK_HIP(launch_init_omega<T>((const T *)omega0[1 - m], p, sh.Gr, sh.Gc, sh.nr_max, ox[m],
                                    odx[m], out + 4, stream));
        CK_HIP(launch_init_publish<T>(W[m], p, sh.Gr, sh.nr_max, pc[m], pd[m], stream));
    }

    SweepParams<T> P[2];
    for (int m = 0; m < 2; ++m) {
        SweepParams<T> &Q = P[m];
        memset(&Q, 0, sizeof(Q));
        Q.S = S[m];
        Q.sd = sd[m];
        Q.W = W[m];
        Q.omp = omp[m];
        Q.omdp = omdp[m];
        Q.pc = pc[m];
        Q.pd = pd[m];
        Q.flags = flags;
        Q.red = red;
        Q.out = out;
        Q.p = p;
        Q.Gr = sh.Gr;
        Q.Gc = sh.Gc;
        Q.maxit = maxit;
        Q.w_lds = sh.w_lds;
        Q.nr_max = sh.nr_max;
        Q.nc_max = sh.nc_max;
        Q.depth = sh.depth;
        Q.rpt = sh.rpt;
        set_overlap(Q, sh.threads, (size_t)max_shared_per_block());
        if (opts && opts->sync_rewrites)
            Q.ovl = 0;
        Q.lam = (T)lam1;
        Q.tol = (T)tol;
        Q.tol_coef = (sizeof(T) == 4) ? T(16.0 * 1.1920928955078125e-07) : T(0);
        Q.spin_limit = kSpinLimit;
        Q.jo_S = S[1 - m];
        Q.jo_sd = sd[1 - m];
        Q.jo_pc = pc[1 - m];
        Q.jo_pd = pd[1 - m];
        Q.jo_omp = ox[m];
        Q.jo_omdp = odx[m];
        Q.lam2 = (T)lam2;
        Q.pop = m;
    }
    CK_HIP(hipEventRecord(ev[4], stream));
    CK_HIP(launch_sweep_joint<T>(P[0], P[1], sh.threads, stream));
    CK_HIP(hipEventRecord(ev[5], stream));
    for (int m = 0; m < 2; ++m)
        CK_HIP(launch_finalize<T>(omp[m], omdp[m], sh.Gr, sh.Gc, sh.nr_max, W[m], p, (T)lam1,
                                  (T *)omega[m], acc + m, cnt + m, out + 4, stream));
    CK_HIP(launch_joint_summary<T>((const T *)omega[0], (const T *)omega[1], p, (T)lam2, acc + 2,
                                   cnt + 2, stream));
    CK_HIP(hipEventRecord(ev[1], stream));

    int hout[kOutWords];
    double hacc[8];
    std::vector<unsigned long long> hred(4 * (size_t)maxit);
    CK_HIP(hipMemcpyAsync(hout, out, sizeof(hout), hipMemcpyDeviceToHost, stream));
    CK_HIP(hipMemcpyAsync(hacc, acc, sizeof(hacc), hipMemcpyDeviceToHost, stream));
    CK_HIP(hipMemcpyAsync(hred.data(), red, sizeof(unsigned long long) * hred.size(),
                          hipMemcpyDeviceToHost, stream));
    CK_HIP(hipStreamSynchronize(stream));
    unsigned long long hcnt[4];
    memcpy(hcnt, hacc + 4, sizeof(hcnt));
    float ms = 0.f, ms_gram = 0.f, ms_sweep = 0.f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (kind == CONCORD_INPUT_Y)
        (void)hipEventElapsedTime(&ms_gram, ev[2], ev[3]);
    (void)hipEventElapsedTime(&ms_sweep, ev[4], ev[5]);

    auto bits_to = [](unsigned long long u) -> double {
        if (sizeof(T) == 8) {
            double d;
            memcpy(&d, &u, 8);
            return d;
        }
        uint32_t w = (uint32_t)u;
        float f;
        memcpy(&f, &w, 4);
        return (double)f;
    };
    const int sweeps = hout[0];
    double *trace = opts ? opts->delta_trace : nullptr;
    int64_t moved = 0, moved_d = 0;
    for (int t = 0; t < sweeps && t < maxit; ++t) {
        if (trace)
            trace[t] = bits_to(hred[4 * (size_t)t]);
        moved += (int64_t)hred[4 * (size_t)t + 2];
        moved_d += (int64_t)hred[4 * (size_t)t + 3];
    }
    const double delta = sweeps > 0 ? bits_to(hred[4 * (size_t)(sweeps - 1)]) : 0.0;
    const double gmax = sweeps > 0 ? bits_to(hred[4 * (size_t)(sweeps - 1) + 1]) : 0.0;
    const double tol_eff = std::max(tol, (double)P[0].tol_coef * gmax);
    int status;
    if (hout[4] & kErrNotPD)
        status = CONCORD_ENOTPD;
    else if (hout[4] & kErrNonFinite)
        status = CONCORD_ENONFINITE;
    else if (hout[2] || hout[3])
        status = CONCORD_EDEVICE;
    else
        status = hout[1] ? CONCORD_OK : CONCORD_NOT_CONVERGED;
    if (info) {
        memset(info, 0, sizeof(*info));
        info->sweeps = sweeps;
        info->status = status;
        info->delta = delta;
        info->tol_eff = tol_eff;
        info->nnz_upper[0] = (int64_t)hcnt[0];
        info->nnz_upper[1] = (int64_t)hcnt[1];
        info->differ_upper = (int64_t)hcnt[2];
        info->objective = hacc[0] + hacc[1] + hacc[2];
        info->elapsed_ms = ms;
        info->gram_ms = ms_gram;
        info->sweep_ms = ms_sweep;
        info->moved_pairs = moved;
        info->moved_diag = moved_d;
        info->row_groups = sh.Gr;
        info->col_slices = sh.Gc;
        info->w_in_lds = sh.w_lds;
        info->block_threads = sh.threads;
        info->pending_depth = sh.depth;
    }
    return status;
}

int validate(concord_input kind, const void *X, int64_t n, int64_t p, double lambda, double tol,
             int32_t maxit, concord_dtype dt, void *omega)
{
    if (!X || !omega)
        return CONCORD_EINVAL;
    if (kind != CONCORD_INPUT_S && kind != CONCORD_INPUT_Y)
        return CONCORD_EINVAL;
    if (dt != CONCORD_F32 && dt != CONCORD_F64)
        return CONCORD_EINVAL;
    if (p < 1 || p > 46340)  // p * p must index as int64 and rows as int32
        return CONCORD_EINVAL;
    if (kind == CONCORD_INPUT_Y && (n < 1 || n > INT32_MAX))
        return CONCORD_EINVAL;
    if (!(lambda >= 0.0) || !isfinite(lambda))
        return CONCORD_EINVAL;
    if (!(tol > 0.0) || !isfinite(tol))
        return CONCORD_EINVAL;
    if (maxit < 1)
        return CONCORD_EINVAL;
    return CONCORD_OK;
}

}  // namespace
}  // namespace concord

using namespace concord;

extern "C" int concord_fit_ex(concord_input kind, const void *X, int64_t n, int64_t p,
                              double lambda, double tol, int32_t maxit, concord_dtype dt,
                              const void *omega0, void *omega, concord_info *info, void *stream,
                              const concord_options *opts)
{
    int rc = validate(kind, X, n, p, lambda, tol, maxit, dt, omega);
    if (rc) {
        if (info) {
            memset(info, 0, sizeof(*info));
            info->status = rc;
        }
        return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    if (dt == CONCORD_F64)
        return fit_impl<double>(kind, X, n, p, lambda, tol, maxit, omega0, omega, info, st, opts);
    return fit_impl<float>(kind, X, n, p, lambda, tol, maxit, omega0, omega, info, st, opts);
}

extern "C" int concord_fit(concord_input kind, const void *X, int64_t n, int64_t p, double lambda,
                           double tol, int32_t maxit, concord_dtype dt, const void *omega0,
                           void *omega, concord_info *info, void *stream)
{
    return concord_fit_ex(kind, X, n, p, lambda, tol, maxit, dt, omega0, omega, info, stream,
                          nullptr);
}

extern "C" int concord_fit_noalloc(concord_input kind, const void *X, int64_t n, int64_t p,
                                   double lambda, double tol, int32_t maxit, concord_dtype dt,
                                   const void *omega0, void *omega, concord_info *info,
                                   void *stream)
{
    int rc = validate(kind, X, n, p, lambda, tol, maxit, dt, omega);
    void *ws = nullptr;
    if (!rc)
        rc = scratch_address(&ws);
    if (rc) {
        if (info) {
            memset(info, 0, sizeof(*info));
            info->status = rc;
        }
        return rc;
    }
    if (info)
        memset(info, 0, sizeof(*info));  // an early error return leaves only the status
    hipStream_t st = (hipStream_t)stream;
    const size_t cap = CONCORD_NOALLOC_SCRATCH_BYTES;
    rc = (dt == CONCORD_F64)
             ? fit_impl<double>(kind, X, n, p, lambda, tol, maxit, omega0, omega, info, st,
                                nullptr, ws, cap)
             : fit_impl<float>(kind, X, n, p, lambda, tol, maxit, omega0, omega, info, st,
                               nullptr, ws, cap);
    if (rc < 0 && info && info->status == 0)
        info->status = rc;
    return rc;
}

extern "C" int concord_fit_joint_ex(concord_input kind, const void *X1, const void *X2,
                                    int64_t n1, int64_t n2, int64_t p, double lambda1,
                                    double lambda2, double tol, int32_t maxit, concord_dtype dt,
                                    const void *omega0_1, const void *omega0_2, void *omega1,
                                    void *omega2, concord_joint_info *info, void *stream,
                                    const concord_options *opts)
{
    int rc = validate(kind, X1, n1, p, lambda1, tol, maxit, dt, omega1);
    if (!rc)
        rc = validate(kind, X2, n2, p, lambda2, tol, maxit, dt, omega2);
    if (!rc && omega1 == omega2)
        rc = CONCORD_EINVAL;
    if (rc) {
        if (info) {
            memset(info, 0, sizeof(*info));
            info->status = rc;
        }
        return rc;
    }
    const void *const X[2] = {X1, X2};
    const int64_t n[2] = {n1, n2};
    const void *const o0[2] = {omega0_1, omega0_2};
    void *const om[2] = {omega1, omega2};
    hipStream_t st = (hipStream_t)stream;
    if (dt == CONCORD_F64)
        return joint_impl<double>(kind, X, n, p, lambda1, lambda2, tol, maxit, o0, om, info, st,
                                  opts);
    return joint_impl<float>(kind, X, n, p, lambda1, lambda2, tol, maxit, o0, om, info, st, opts);
}

extern "C" int concord_fit_joint(concord_input kind, const void *X1, const void *X2, int64_t n1,
                                 int64_t n2, int64_t p, double lambda1, double lambda2,
                                 double tol, int32_t maxit, concord_dtype dt,
                                 const void *omega0_1, const void *omega0_2, void *omega1,
                                 void *omega2, concord_joint_info *info, void *stream)
{
    return concord_fit_joint_ex(kind, X1, X2, n1, n2, p, lambda1, lambda2, tol, maxit, dt,
                                omega0_1, omega0_2, omega1, omega2, info, stream, nullptr);
}

extern "C" int concord_fit_batched_ex(int32_t B, concord_input kind, const void *const *X,
                                      const int64_t *n, const int64_t *p, int32_t L,
                                      const double *lambdas, double tol, int32_t maxit,
                                      concord_dtype dt, void *const *omega, concord_info *info,
                                      void *stream, const concord_batch_options *opts)
{
    if (B < 1 || L < 1 || !X || !p || !lambdas || !omega || (kind == CONCORD_INPUT_Y && !n) ||
        (long long)L * maxit > (1ll << 24))
        return CONCORD_EINVAL;
    for (int b = 0; b < B; ++b) {
        for (int l = 0; l < L; ++l) {
            int rc = validate(kind, X[b], n ? n[b] : 1, p[b], lambdas[(size_t)b * L + l], tol,
                              maxit, dt, omega[(size_t)b * L + l]);
            if (rc)
                return rc;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    if (dt == CONCORD_F64)
        return batched_impl<double>(B, kind, X, n, p, L, lambdas, tol, maxit, omega, info, st,
                                    opts);
    return batched_impl<float>(B, kind, X, n, p, L, lambdas, tol, maxit, omega, info, st, opts);
}

extern "C" int concord_fit_batched(int32_t B, concord_input kind, const void *const *X,
                                   const int64_t *n, const int64_t *p, int32_t L,
                                   const double *lambdas, double tol, int32_t maxit,
                                   concord_dtype dt, void *const *omega, concord_info *info,
                                   void *stream)
{
    return concord_fit_batched_ex(B, kind, X, n, p, L, lambdas, tol, maxit, dt, omega, info,
                                  stream, nullptr);
}

extern "C" int concord_backward_ex(const void *S, const void *omega_hat, int64_t p,
                                   const void *grad_omega, void *grad_S, double *grad_lambda,
                                   double tol, int32_t maxit, concord_dtype dt, concord_info *info,
                                   void *stream, const concord_options *opts)
{
    int rc = CONCORD_OK;
    if (!S || !omega_hat || !grad_omega || !grad_S)
        rc = CONCORD_EINVAL;
    else
        rc = validate(CONCORD_INPUT_S, S, 1, p, 0.0, tol, maxit, dt, grad_S);
    if (rc) {
        if (info) {
            memset(info, 0, sizeof(*info));
            info->status = rc;
        }
        return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    if (dt == CONCORD_F64)
        return backward_impl<double>(S, omega_hat, p, grad_omega, grad_S, grad_lambda, tol, maxit,
                                     info, st, opts);
    return backward_impl<float>(S, omega_hat, p, grad_omega, grad_S, grad_lambda, tol, maxit,
                                info, st, opts);
}

extern "C" int concord_backward(const void *S, const void *omega_hat, int64_t p,
                                const void *grad_omega, void *grad_S, double *grad_lambda,
                                double tol, int32_t maxit, concord_dtype dt, concord_info *info,
                                void *stream)
{
    return concord_backward_ex(S, omega_hat, p, grad_omega, grad_S, grad_lambda, tol, maxit, dt,
                               info, stream, nullptr);
}

extern "C" int concord_gram(const void *Y, int64_t n, int64_t p, concord_dtype dt, void *S,
                            void *stream)
{
    if (!Y || !S || n < 1 || n > INT32_MAX || p < 1 || p > 46340)
        return CONCORD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (dt == CONCORD_F64)
        e = launch_gram<double>((const double *)Y, (int)n, (int)p, (double *)S, st);
    else if (dt == CONCORD_F32)
        e = launch_gram<float>((const float *)Y, (int)n, (int)p, (float *)S, st);
    else
        return CONCORD_EINVAL;
    if (e != hipSuccess)
        return map_hip(e);
    return map_hip(hipStreamSynchronize(st));
}

extern "C" int64_t concord_schedule(int64_t p, int32_t *pairs)
{
    if (p < 1 || p > 46340 || !pairs)
        return CONCORD_EINVAL;
    const Circle C = Circle::make((int)p);
    for (int r = 0; r < C.m; ++r)
        for (int q = 0; q < C.H; ++q) {
            int a, b;
            C.pair(r, q, &a, &b);
            pairs[((size_t)r * C.H + q) * 2 + 0] = a;
            pairs[((size_t)r * C.H + q) * 2 + 1] = b;
        }
    return C.m;
}

extern "C" const char *concord_strerror(int code)
{
    switch (code) {
    case CONCORD_OK: return "converged";
    case CONCORD_NOT_CONVERGED: return "sweep limit reached before the tolerance (last iterate returned)";
    case CONCORD_EINVAL: return "invalid argument";
    case CONCORD_ENONFINITE: return "non-finite value in the input or the iteration";
    case CONCORD_ENOTPD: return "a diagonal entry of S is not positive";
    case CONCORD_ENOMEM: return "device workspace allocation failed";
    case CONCORD_EDEVICE: return "HIP runtime error or a device wait exceeded its bound";
    case CONCORD_ELAUNCH: return "launch shape cannot be made co-resident on this device";
    case CONCORD_ESCRATCH:
        return "the solve needs more workspace than concord_fit_noalloc's fixed scratch "
               "(CONCORD_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown status code";
    }
}

extern "C" const char *concord_version(void) { return "concord-mi355x 0.1.0 (gfx950)"; }
