// concord_bench: native driver for profiling one or more CONCORD-PCD solves
// through the C ABI, with no Python in the process (for rocprofv3 runs).
//
//   concord_bench --y FILE --n N --p P [--lam L] [--tol T] [--maxit K]
//                 [--reps R] [--f32] [--row-groups A] [--col-slices B]
//                 [--threads C] [--depth D]
//   concord_bench --copy MIB
//   concord_bench --y FILE --y2 FILE2 --lam2 L2 --n N --p P [...]
//
// --copy runs one device-to-device copy of MIB mebibytes (the runtime's copy
// kernel) and exits: a reference of known size for hardware byte counters.
//
// FILE holds Y as raw little-endian float64, n x p row-major (bench.py
// --dump-y writes it).  Y is copied to the device once; each repetition is
// one concord_fit from Y.  One JSON line per repetition goes to stdout.
// With --y2, each repetition is one concord_fit_joint of the two populations
// Y (FILE) and Y2 (FILE2, also n x p) with thresholds --lam and --lam2.
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
                 "[--depth D] [--y2 FILE2 --lam2 L2]\n       concord_bench --copy MIB\n");
}

}  // namespace

int main(int argc, char **argv)
{
    std::string path, path2;
    double lam2 = 0.0;
    long long n = 0, p = 0, copy_mib = 0;
    double lam = 0.1, tol = 1e-6;
    int maxit = 500, reps = 1, f32 = 0;
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
                    "\"row_groups\": %d, \"col_slices\": %d, \"threads\": %d, \"depth\": %d}\n",
                    r, rc, info.sweeps, info.delta, (long long)info.nnz_upper, info.elapsed_ms,
                    info.gram_ms, info.sweep_ms, (long long)info.moved_pairs,
                    (long long)info.moved_diag, info.row_groups, info.col_slices,
                    info.block_threads, info.pending_depth);
        std::fflush(stdout);
        if (rc < 0)
            break;
    }
    (void)hipFree(dY);
    (void)hipFree(dOm);
    return rc < 0 ? 1 : 0;
}
