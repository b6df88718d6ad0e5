// Support kernels of the active-set sweeps: the support of the current Omega
// as an edge list (to be coloured), the dense Omega back from the sweep
// layout of a colour table, and the refresh of Algorithm 1's layout after
// the sweeps over that table.
#include "device_common.hpp"
#include "schedule.hpp"
#include "support.hpp"

namespace concord {

namespace {

constexpr int kThreads = 256;

inline int grid_for(long long work, int cap = 4096)
{
    long long g = (work + kThreads - 1) / kThreads;
    if (g < 1)
        g = 1;
    return (int)(g > cap ? cap : g);
}

// Pairs i < j with omega_ij != 0, appended to edges[2 e], edges[2 e + 1]
// (order unspecified; *count ends as the number found, even past cap).
template <typename T>
__global__ void support_edges_kernel(const T *__restrict__ omega, int p, int *__restrict__ count,
                                     int *__restrict__ edges, long long cap)
{
    const long long total = (long long)p * p;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / p), j = (int)(e - (long long)i * p);
        if (j > i && omega[e] != T(0)) {
            const int slot = atomicAdd(count, 1);
            if (slot < cap) {
                edges[2 * (long long)slot] = i;
                edges[2 * (long long)slot + 1] = j;
            }
        }
    }
}

__global__ void fill_int_kernel(int *__restrict__ x, long long n, int v)
{
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        x[e] = v;
}

// Each edge writes its two table entries; a colour's edges share no vertex,
// so every entry is written at most once.
__global__ void partner_table_kernel(const int *__restrict__ edges, const int *__restrict__ colour,
                                     int ne, int p, int *__restrict__ part)
{
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = edges[2 * e], j = edges[2 * e + 1];
        const long long row = (long long)colour[e] * p;
        part[row + i] = j;
        part[row + j] = i;
    }
}

// Dense Omega from the copies of column slice 0: omega_ij at colour r of
// row i's table entry, omega_ii per row.  Entries in no colour stay 0.
template <typename T>
__global__ void scatter_omega_kernel(const T *__restrict__ omp, const T *__restrict__ omdp,
                                     const int *__restrict__ part, int mt, int Gr, int Gc, int NR,
                                     int p, T *__restrict__ omega)
{
    const long long total = (long long)Gr * (mt + 1) * NR;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long per = (long long)(mt + 1) * NR;
        const int a = (int)(e / per);
        const long long rem = e - (long long)a * per;
        const int r = (int)(rem / NR), k = (int)(rem - (long long)r * NR);
        const int i = a + k * Gr;
        if (i >= p)
            continue;
        const int g = a * Gc;
        if (r == mt) {
            omega[(size_t)i * p + i] = omdp[(size_t)g * NR + k];
        } else {
            const int j = part[(size_t)r * p + i];
            if (j >= 0)
                omega[(size_t)i * p + j] = omp[((size_t)g * mt + r) * NR + k];
        }
    }
}

// Algorithm 1's sweep layout after sweeps over a colouring of the support:
// only the listed support pairs and the diagonal can have changed, so only
// their entries are rewritten, in the copy of every column slice.  Work item
// e < 2 ne Gc is endpoint e / Gc % 2 of edge e / (2 Gc) in slice e % Gc;
// the next p Gc items are the diagonals.
template <typename T>
__global__ void refresh_layout_kernel(const T *__restrict__ omega, const int *__restrict__ edges,
                                      int ne, int p, int Gr, int Gc, int NR,
                                      T *__restrict__ omp, T *__restrict__ omdp)
{
    const Circle C = Circle::make(p);
    const long long ne_work = 2ll * ne * Gc, total = ne_work + (long long)p * Gc;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < ne_work) {
            const int b = (int)(e % Gc);
            const long long q = e / Gc;
            const int side = (int)(q & 1);
            const long long ed = q >> 1;
            const int i = edges[2 * ed + side], j = edges[2 * ed + 1 - side];
            const int a = i % Gr, k = i / Gr, g = a * Gc + b;
            omp[((size_t)g * C.m + C.colour(i, j)) * NR + k] = omega[(size_t)i * p + j];
        } else {
            const long long d = e - ne_work;
            const int b = (int)(d % Gc), i = (int)(d / Gc);
            const int a = i % Gr, k = i / Gr, g = a * Gc + b;
            omdp[(size_t)g * NR + k] = omega[(size_t)i * p + i];
        }
    }
}

}  // namespace

template <typename T>
hipError_t launch_refresh_layout(const T *omega, const int *edges, int ne, int p, int Gr, int Gc,
                                 int NR, T *omp, T *omdp, hipStream_t st)
{
    const long long work = 2ll * ne * Gc + (long long)p * Gc;
    hipLaunchKernelGGL(refresh_layout_kernel<T>, dim3(grid_for(work, 4096)), dim3(kThreads), 0, st,
                       omega, edges, ne, p, Gr, Gc, NR, omp, omdp);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_support_edges(const T *omega, int p, int *count, int *edges, long long cap,
                                hipStream_t st)
{
    hipLaunchKernelGGL(support_edges_kernel<T>, dim3(grid_for((long long)p * p, 4096)),
                       dim3(kThreads), 0, st, omega, p, count, edges, cap);
    return hipGetLastError();
}

hipError_t launch_partner_table(const int *edges, const int *colour, int ne, int p, int m,
                                int *part, hipStream_t st)
{
    const long long n = (long long)m * p;
    hipLaunchKernelGGL(fill_int_kernel, dim3(grid_for(n, 4096)), dim3(kThreads), 0, st, part, n,
                       -1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ne <= 0)
        return e;
    hipLaunchKernelGGL(partner_table_kernel, dim3(grid_for(ne, 4096)), dim3(kThreads), 0, st,
                       edges, colour, ne, p, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scatter_omega(const T *omp, const T *omdp, const int *part, int mt, int Gr,
                                int Gc, int NR, int p, T *omega, hipStream_t st)
{
    hipLaunchKernelGGL(scatter_omega_kernel<T>,
                       dim3(grid_for((long long)Gr * (mt + 1) * NR, 4096)), dim3(kThreads), 0, st,
                       omp, omdp, part, mt, Gr, Gc, NR, p, omega);
    return hipGetLastError();
}

#define CONCORD_ACTIVE_INST(T)                                                                   \
    template hipError_t launch_support_edges<T>(const T *, int, int *, int *, long long,        \
                                                hipStream_t);                                    \
    template hipError_t launch_scatter_omega<T>(const T *, const T *, const int *, int, int, int, \
                                                int, int, T *, hipStream_t);                     \
    template hipError_t launch_refresh_layout<T>(const T *, const int *, int, int, int, int, int, \
                                                 T *, T *, hipStream_t);

CONCORD_ACTIVE_INST(float)
CONCORD_ACTIVE_INST(double)

}  // namespace concord
