// concord_bench: native driver for profiling one or more CONCORD-PCD solves
// through the C ABI, with no Python in the process (for rocprofv3 runs).
//
//   concord_bench --y FILE --n N --p P [--lam L] [--tol T] [--maxit K]
//                 [--reps R] [--f32] [--row-groups A] [--col-slices B]
//                 [--threads C] [--depth D] [--active [--active-maxit K]]
//   concord_bench --copy MIB
//   concord_bench --y FILE --y2 FILE2 --lam2 L2 --n N --p P [...]
//   concord_bench --batched DIR [--plan FILE] [--tol T] [--maxit K] [--reps R]
//                 [--threads C] [--cpl K] [--depth D] [--sync-rewrites]
//   concord_bench --backward --y FILE --n N --p P [--lam L] [--tol T] [--reps R]
//
// With both --y and --batched, the single solves run first and then one
// repetition of the batch (tol 1e-5, maxit 500), in one process.
//
// Runs joined by --then (each written as above) are made in order in one
// process; the first one that fails ends the process with its status.
//
// --copy runs one device-to-device copy of MIB mebibytes (the runtime's copy
// kernel) and exits: a reference of known size for hardware byte counters.
//
// FILE holds Y as raw little-endian float64, n x p row-major (bench.py
// --dump-y writes it).  Y is copied to the device once; each repetition is
// one concord_fit from Y.  One JSON line per repetition goes to stdout.
// With --y2, each repetition is one concord_fit_joint of the two populations
// Y (FILE) and Y2 (FILE2, also n x p) with thresholds --lam and --lam2.
// With --batched, DIR holds problems.txt ('p n' per problem), lambdas.txt
// and y_<b>.bin (raw float64 n x p), as bench.py --dump-batched writes them;
// each repetition is one FP32 concord_fit_batched_ex of all problems along
// the lambda path, with the workgroup plan of --plan FILE (one line per
// problem: its workgroups, optionally followed by its column slices) or the
// built-in plan; --threads and --cpl set the batch's threads per workgroup
// and columns per lane in row rewrites.  With --backward, each repetition is one
// FP64 solve from Y followed by concord_backward of
// L = |Omega-hat - Omega_0|_F^2 with the chain Omega_0 (1 on the diagonal,
// 0.4 beside it), the gradient workload of bench.py.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/concord.h"

namespace {

void usage()
{
    std::fprintf(stderr,
                 "usage: concord_bench --y FILE --n N --p P [--lam L] [--tol T] [--maxit K] "
                 "[--reps R] [--f32] [--row-groups A] [--col-slices B] [--threads C] "
                 "[--depth D] [--active [--active-maxit K]] [--y2 FILE2 --lam2 L2] "
                 "[--sync-rewrites]\n"
                 "       concord_bench --copy MIB\n"
                 "       concord_bench --batched DIR [--plan FILE] [--tol T] [--maxit K] "
                 "[--reps R] [--threads C] [--cpl K] [--depth D]\n"
                 "       concord_bench --backward --y FILE --n N --p P [--lam L] [--tol T] "
                 "[--reps R]\n"
                 "       concord_bench RUN --then RUN [--then RUN ...]\n");
}

// The batched workload from DIR, FP32, one launch per repetition.
int run_batched(const std::string &dir, const std::string &plan, double tol, int maxit, int reps,
                int threads, int cpl, int sync_rw, int depth)
{
    std::vector<int64_t> ps, ns;
    {
        FILE *f = std::fopen((dir + "/problems.txt").c_str(), "r");
        long long a = 0, b = 0;
        while (f && std::fscanf(f, "%lld %lld", &a, &b) == 2) {
            ps.push_back(a);
            ns.push_back(b);
        }
        if (f)
            std::fclose(f);
    }
    std::vector<double> lams;
    {
        FILE *f = std::fopen((dir + "/lambdas.txt").c_str(), "r");
        double x = 0;
        while (f && std::fscanf(f, "%lf", &x) == 1)
            lams.push_back(x);
        if (f)
            std::fclose(f);
    }
    const int B = (int)ps.size(), L = (int)lams.size();
    if (B < 1 || L < 1) {
        std::fprintf(stderr, "concord_bench: no problems or lambdas in %s\n", dir.c_str());
        return 1;
    }
    std::vector<int32_t> pw, pc;
    bool any_slices = false;
    if (!plan.empty()) {
        FILE *f = std::fopen(plan.c_str(), "r");
        char line[256];
        while (f && std::fgets(line, sizeof(line), f)) {
            int g = 0, c = 1;
            const int got = std::sscanf(line, "%d %d", &g, &c);
            if (got < 1)
                continue;
            pw.push_back(g);
            pc.push_back(got >= 2 ? c : 1);
            any_slices = any_slices || got >= 2;
        }
        if (f)
            std::fclose(f);
        if ((int)pw.size() != B) {
            std::fprintf(stderr, "concord_bench: %s holds %zu counts for %d problems\n",
                         plan.c_str(), pw.size(), B);
            return 1;
        }
    }
    std::vector<void *> dX(B, nullptr), dOm((size_t)B * L, nullptr);
    std::vector<double> lam_all((size_t)B * L);
    for (int b = 0; b < B; ++b) {
        const size_t cnt = (size_t)ns[b] * ps[b];
        std::vector<double> y(cnt);
        const std::string file = dir + "/y_" + std::to_string(b) + ".bin";
        FILE *f = std::fopen(file.c_str(), "rb");
        if (!f || std::fread(y.data(), sizeof(double), cnt, f) != cnt) {
            std::fprintf(stderr, "concord_bench: cannot read %s\n", file.c_str());
            return 1;
        }
        std::fclose(f);
        std::vector<float> y32(y.begin(), y.end());
        if (hipMalloc(&dX[b], sizeof(float) * cnt) != hipSuccess ||
            hipMemcpy(dX[b], y32.data(), sizeof(float) * cnt, hipMemcpyHostToDevice) !=
                hipSuccess) {
            std::fprintf(stderr, "concord_bench: device allocation or copy failed\n");
            return 1;
        }
        for (int l = 0; l < L; ++l) {
            if (hipMalloc(&dOm[(size_t)b * L + l], sizeof(float) * ps[b] * ps[b]) != hipSuccess) {
                std::fprintf(stderr, "concord_bench: device allocation failed\n");
                return 1;
            }
            lam_all[(size_t)b * L + l] = lams[l];
        }
    }
    concord_batch_options bo;
    std::memset(&bo, 0, sizeof(bo));
    bo.problem_workgroups = pw.empty() ? nullptr : pw.data();
    bo.problem_col_slices = any_slices ? pc.data() : nullptr;
    bo.block_threads = threads;
    bo.cols_per_lane = cpl;
    bo.pending_depth = depth;
    bo.sync_rewrites = sync_rw;
    std::vector<concord_info> info((size_t)B * L);
    int rc = 0;
    for (int r = 0; r < reps; ++r) {
        rc = concord_fit_batched_ex(B, CONCORD_INPUT_Y, dX.data(), ns.data(), ps.data(), L,
                                    lam_all.data(), tol, maxit, CONCORD_F32, dOm.data(),
                                    info.data(), nullptr, &bo);
        long long sweeps = 0;
        double dev_max = 0.0;
        for (int b = 0; b < B; ++b) {
            double dev = 0.0;
            for (int l = 0; l < L; ++l) {
                sweeps += info[(size_t)b * L + l].sweeps;
                dev += info[(size_t)b * L + l].sweep_ms;
            }
            dev_max = dev > dev_max ? dev : dev_max;
        }
        std::printf("{\"rep\": %d, \"code\": %d, \"problems\": %d, \"lambdas\": %d, "
                    "\"plan\": \"%s\", \"elapsed_ms\": %.3f, \"sweeps_total\": %lld, "
                    "\"slowest_problem_ms\": %.3f}\n",
                    r, rc, B, L, pw.empty() ? "built-in" : "file", info[0].elapsed_ms, sweeps,
                    dev_max);
        std::fflush(stdout);
        if (rc < 0)
            break;
    }
    for (void *x : dX)
        (void)hipFree(x);
    for (void *x : dOm)
        (void)hipFree(x);
    return rc < 0 ? 1 : 0;
}

}  // namespace

int run(int argc, char **argv)
{
    std::string path, path2, bdir, plan;
    double lam2 = 0.0;
    int backward = 0;
    long long n = 0, p = 0, copy_mib = 0;
    double lam = 0.1, tol = 1e-6;
    int maxit = 500, reps = 1, f32 = 0, cpl = 0;
    concord_options opt;
    std::memset(&opt, 0, sizeof(opt));
    for (int k = 1; k < argc; ++k) {
        std::string a = argv[k];
        auto next = [&]() -> const char * {
            if (k + 1 >= argc) {
                usage();
                std::exit(2);
            }
            return argv[++k];
        };
        if (a == "--y")
            path = next();
        else if (a == "--n")
            n = std::atoll(next());
        else if (a == "--p")
            p = std::atoll(next());
        else if (a == "--lam")
            lam = std::atof(next());
        else if (a == "--tol")
            tol = std::atof(next());
        else if (a == "--maxit")
            maxit = std::atoi(next());
        else if (a == "--reps")
            reps = std::atoi(next());
        else if (a == "--f32")
            f32 = 1;
        else if (a == "--row-groups")
            opt.row_groups = std::atoi(next());
        else if (a == "--col-slices")
            opt.col_slices = std::atoi(next());
        else if (a == "--threads")
            opt.block_threads = std::atoi(next());
        else if (a == "--depth")
            opt.pending_depth = std::atoi(next());
        else if (a == "--active")
            opt.active_set = 1;
        else if (a == "--active-maxit")
            opt.active_maxit = std::atoi(next());
        else if (a == "--backward")
            backward = 1;
        else if (a == "--batched")
            bdir = next();
        else if (a == "--plan")
            plan = next();
        else if (a == "--cpl")
            cpl = std::atoi(next());
        else if (a == "--sync-rewrites")
            opt.sync_rewrites = 1;
        else if (a == "--y2")
            path2 = next();
        else if (a == "--lam2")
            lam2 = std::atof(next());
        else if (a == "--copy")
            copy_mib = std::atoll(next());
        else {
            usage();
            return 2;
        }
    }
    if (copy_mib > 0) {
        const size_t bytes = (size_t)copy_mib << 20;
        void *src = nullptr, *dst = nullptr;
        if (hipMalloc(&src, bytes) != hipSuccess || hipMalloc(&dst, bytes) != hipSuccess ||
            hipMemset(src, 1, bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(dst, src, bytes, hipMemcpyDeviceToDevice) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess) {
            std::fprintf(stderr, "concord_bench: copy failed\n");
            return 1;
        }
        std::printf("{\"copy_bytes\": %zu}\n", bytes);
        (void)hipFree(src);
        (void)hipFree(dst);
        return 0;
    }
    if (!bdir.empty() && path.empty())
        return run_batched(bdir, plan, tol, maxit, reps, opt.block_threads, cpl,
                           opt.sync_rewrites, opt.pending_depth);
    if (path.empty() || n < 1 || p < 1 || reps < 1) {
        usage();
        return 2;
    }
    const size_t esz = f32 ? 4 : 8;
    // reads an n x p float64 file and copies it to the device in the solve's type
    auto upload = [&](const std::string &file, void **dev) -> bool {
        std::vector<double> y((size_t)n * p);
        FILE *f = std::fopen(file.c_str(), "rb");
        if (!f || std::fread(y.data(), sizeof(double), y.size(), f) != y.size()) {
            std::fprintf(stderr, "concord_bench: cannot read %zu doubles from %s\n", y.size(),
                         file.c_str());
            if (f)
                std::fclose(f);
            return false;
        }
        std::fclose(f);
        std::vector<float> y32;
        const void *host = y.data();
        if (f32) {
            y32.assign(y.begin(), y.end());
            host = y32.data();
        }
        if (hipMalloc(dev, esz * y.size()) != hipSuccess ||
            hipMemcpy(*dev, host, esz * y.size(), hipMemcpyHostToDevice) != hipSuccess) {
            std::fprintf(stderr, "concord_bench: device allocation or copy failed\n");
            return false;
        }
        return true;
    };
    void *dY = nullptr, *dOm = nullptr, *dY2 = nullptr, *dOm2 = nullptr;
    if (!upload(path, &dY) || hipMalloc(&dOm, esz * (size_t)p * p) != hipSuccess) {
        std::fprintf(stderr, "concord_bench: set-up failed\n");
        return 1;
    }
    if (backward) {
        if (f32) {
            std::fprintf(stderr, "concord_bench: --backward runs in FP64\n");
            return 2;
        }
        const size_t pp = (size_t)p * p;
        void *dS = nullptr, *dC = nullptr, *dG = nullptr;
        if (hipMalloc(&dS, 8 * pp) != hipSuccess || hipMalloc(&dC, 8 * pp) != hipSuccess ||
            hipMalloc(&dG, 8 * pp) != hipSuccess ||
            concord_gram(dY, n, p, CONCORD_F64, dS, nullptr) != CONCORD_OK) {
            std::fprintf(stderr, "concord_bench: set-up failed\n");
            return 1;
        }
        std::vector<double> om(pp), c(pp);
        int rc = 0;
        for (int r = 0; r < reps; ++r) {
            concord_info fi, bi;
            rc = concord_fit(CONCORD_INPUT_S, dS, n, p, lam, tol, maxit, CONCORD_F64, nullptr,
                             dOm, &fi, nullptr);
            if (rc < 0)
                break;
            // C = dL/dOmega-hat = 2 (Omega-hat - Omega_0), chain Omega_0
            if (hipMemcpy(om.data(), dOm, 8 * pp, hipMemcpyDeviceToHost) != hipSuccess)
                return 1;
            for (long long i = 0; i < p; ++i)
                for (long long j = 0; j < p; ++j) {
                    const double o0 = (i == j) ? 1.0 : ((i - j == 1 || j - i == 1) ? 0.4 : 0.0);
                    c[(size_t)i * p + j] = 2.0 * (om[(size_t)i * p + j] - o0);
                }
            if (hipMemcpy(dC, c.data(), 8 * pp, hipMemcpyHostToDevice) != hipSuccess)
                return 1;
            double gl = 0.0;
            rc = concord_backward(dS, dOm, p, dC, dG, &gl, tol, maxit, CONCORD_F64, &bi, nullptr);
            std::printf("{\"rep\": %d, \"code\": %d, \"forward_ms\": %.3f, \"forward_sweeps\": %d, "
                        "\"backward_ms\": %.3f, \"backward_sweeps\": %d, \"grad_lambda\": %.10g}\n",
                        r, rc, fi.elapsed_ms, fi.sweeps, bi.elapsed_ms, bi.sweeps, gl);
            std::fflush(stdout);
            if (rc < 0)
                break;
        }
        (void)hipFree(dS);
        (void)hipFree(dC);
        (void)hipFree(dG);
        (void)hipFree(dY);
        (void)hipFree(dOm);
        return rc < 0 ? 1 : 0;
    }
    if (!path2.empty()) {
        if (!upload(path2, &dY2) || hipMalloc(&dOm2, esz * (size_t)p * p) != hipSuccess) {
            std::fprintf(stderr, "concord_bench: set-up failed\n");
            return 1;
        }
        int rc = 0;
        for (int r = 0; r < reps; ++r) {
            concord_joint_info info;
            rc = concord_fit_joint_ex(CONCORD_INPUT_Y, dY, dY2, n, n, p, lam, lam2, tol, maxit,
                                      f32 ? CONCORD_F32 : CONCORD_F64, nullptr, nullptr, dOm,
                                      dOm2, &info, nullptr, &opt);
            std::printf("{\"rep\": %d, \"code\": %d, \"sweeps\": %d, \"delta\": %.6e, "
                        "\"nnz_upper\": [%lld, %lld], \"differ_upper\": %lld, "
                        "\"elapsed_ms\": %.3f, \"gram_ms\": %.3f, \"sweep_ms\": %.3f, "
                        "\"moved_pairs\": %lld, \"moved_diag\": %lld, \"row_groups\": %d, "
                        "\"col_slices\": %d, \"threads\": %d, \"depth\": %d}\n",
                        r, rc, info.sweeps, info.delta, (long long)info.nnz_upper[0],
                        (long long)info.nnz_upper[1], (long long)info.differ_upper,
                        info.elapsed_ms, info.gram_ms, info.sweep_ms,
                        (long long)info.moved_pairs, (long long)info.moved_diag, info.row_groups,
                        info.col_slices, info.block_threads, info.pending_depth);
            std::fflush(stdout);
            if (rc < 0)
                break;
        }
        (void)hipFree(dY);
        (void)hipFree(dOm);
        (void)hipFree(dY2);
        (void)hipFree(dOm2);
        return rc < 0 ? 1 : 0;
    }
    int rc = 0;
    for (int r = 0; r < reps; ++r) {
        concord_info info;
        rc = concord_fit_ex(CONCORD_INPUT_Y, dY, n, p, lam, tol, maxit,
                            f32 ? CONCORD_F32 : CONCORD_F64, nullptr, dOm, &info, nullptr, &opt);
        std::printf("{\"rep\": %d, \"code\": %d, \"sweeps\": %d, \"delta\": %.6e, "
                    "\"nnz_upper\": %lld, \"elapsed_ms\": %.3f, \"gram_ms\": %.3f, "
                    "\"sweep_ms\": %.3f, \"moved_pairs\": %lld, \"moved_diag\": %lld, "
                    "\"row_groups\": %d, \"col_slices\": %d, \"threads\": %d, \"depth\": %d, "
                    "\"active_sweeps\": %d}\n",
                    r, rc, info.sweeps, info.delta, (long long)info.nnz_upper, info.elapsed_ms,
                    info.gram_ms, info.sweep_ms, (long long)info.moved_pairs,
                    (long long)info.moved_diag, info.row_groups, info.col_slices,
                    info.block_threads, info.pending_depth, info.active_sweeps);
        std::fflush(stdout);
        if (rc < 0)
            break;
    }
    (void)hipFree(dY);
    (void)hipFree(dOm);
    if (rc >= 0 && !bdir.empty()) {
        // the batched workload after the single solves, in the same process
        // (one profiler run then covers both kernels), at the batch's own
        // tolerance and sweep limit, one repetition, 512 threads
        return run_batched(bdir, plan, 1e-5, 500, 1, 0, cpl, opt.sync_rewrites, 0);
    }
    return rc < 0 ? 1 : 0;
}

// Before the process ends: wait for every queued operation on the device,
// return the stream-ordered pool's memory, so that nothing the driver or the
// library issued is left for the runtime's exit-time teardown to retire.
int main(int argc, char **argv)
{
    // "--then" separates runs made one after the other in this process, so
    // one profiler run covers several workloads; the first failure ends it
    int rc = 0;
    std::vector<char *> seg{argv[0]};
    for (int k = 1; k <= argc && rc == 0; ++k) {
        if (k < argc && std::strcmp(argv[k], "--then") != 0) {
            seg.push_back(argv[k]);
            continue;
        }
        rc = run((int)seg.size(), seg.data());
        seg.resize(1);
    }
    (void)hipDeviceSynchronize();
    int dev = 0;
    hipMemPool_t pool = nullptr;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess &&
        pool)
        (void)hipMemPoolTrimTo(pool, 0);
    (void)hipDeviceSynchronize();
    return rc;
}
