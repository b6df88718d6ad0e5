// S = Y^T Y / n on matrix cores (Algorithm 1's T = X^T X, on the S scale),
// and the general product C = A^T B used to form W = Omega0 S for a warm start.
//
// Y is n x p row-major.  For the Gram matrix each workgroup computes one
// 64 x 64 tile of S with tile row <= tile column (S is symmetric) and writes
// it and its mirror; for C = A^T B (A: K x M, B: K x N) every tile is computed.
// Four waves split the tile into 2 x 2 quadrants of 32 x 32; each quadrant
// is 2 x 2 MFMA 16x16x4 blocks.  Y panels of 32 k-rows are staged in LDS,
// one for the tile's rows and one for its columns (the same panel on the
// diagonal).
//
// MFMA 16x16x4 operand layout, lane l of the wave (checked on gfx950):
//   A (16 x 4):  A[l % 16][l / 16]      B (4 x 16):  B[l / 16][l % 16]
//   D (16 x 16): result element v of lane l is D[row][l % 16] with
//                row = 4 (l / 16) + v  for f32,   row = l / 16 + 4 v  for f64.
// Here A = Y^T restricted to 16 tile rows and 4 k values, B = Y likewise.
#include <hip/hip_runtime.h>

#include "gram.hpp"

namespace concord {

namespace {

constexpr int TILE = 64;
constexpr int KB = 32;

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    using V4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    __device__ static V4 step(double a, double b, V4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <>
struct Mfma<float> {
    using V4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;
    __device__ static V4 step(float a, float b, V4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

}  // namespace

// SYM: A == B (the Gram matrix), M == N, upper tiles only, mirrored writes.
template <typename T, bool SYM>
__global__ void __launch_bounds__(256) atb_mfma_kernel(const T *__restrict__ A,
                                                       const T *__restrict__ B, int K, int M,
                                                       int N, T scale, T *__restrict__ Cout)
{
    using V4 = typename Mfma<T>::V4;
    __shared__ T As[KB][TILE + 1];
    __shared__ T Bs[KB][TILE + 1];

    int ti, tj;
    if (SYM) {
        // Upper-triangular tile index -> (ti, tj), ti <= tj.
        const int nt = (M + TILE - 1) / TILE;
        int bid = blockIdx.x;
        ti = 0;
        while (bid >= nt - ti) {
            bid -= nt - ti;
            ++ti;
        }
        tj = ti + bid;
    } else {
        ti = blockIdx.y;
        tj = blockIdx.x;
    }
    const int I0 = ti * TILE, J0 = tj * TILE;
    const bool diag = SYM && (ti == tj);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int qi = (wave >> 1) * 32, qj = (wave & 1) * 32;  // quadrant origin in the tile

    V4 acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            for (int v = 0; v < 4; ++v)
                acc[x][y][v] = T(0);

    for (int k0 = 0; k0 < K; k0 += KB) {
        // Stage A[k0 .. k0+KB) x [I0 .. I0+64) and B[k0 .. k0+KB) x [J0 .. J0+64);
        // zero outside the matrices.
        for (int e = tid; e < KB * TILE; e += 256) {
            const int kk = e / TILE, c = e % TILE;
            const int k = k0 + kk;
            T va = T(0), vb = T(0);
            if (k < K) {
                if (I0 + c < M)
                    va = A[(size_t)k * M + I0 + c];
                if (!diag && J0 + c < N)
                    vb = B[(size_t)k * N + J0 + c];
            }
            As[kk][c] = va;
            Bs[kk][c] = diag ? va : vb;
        }
        __syncthreads();
        for (int kk = 0; kk < KB; kk += 4) {
            const int kr = kk + (lane >> 4), cc = lane & 15;
            T fa[2], fb[2];
            for (int x = 0; x < 2; ++x)
                fa[x] = As[kr][qi + 16 * x + cc];
            for (int y = 0; y < 2; ++y)
                fb[y] = Bs[kr][qj + 16 * y + cc];
            for (int x = 0; x < 2; ++x)
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = Mfma<T>::step(fa[x], fb[y], acc[x][y]);
        }
        __syncthreads();
    }

    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            for (int v = 0; v < 4; ++v) {
                const int i = I0 + qi + 16 * x + Mfma<T>::row(lane, v);
                const int j = J0 + qj + 16 * y + (lane & 15);
                if (i < M && j < N) {
                    const T val = acc[x][y][v] * scale;
                    Cout[(size_t)i * N + j] = val;
                    if (SYM && !diag)
                        Cout[(size_t)j * N + i] = val;
                }
            }
}

template <typename T>
hipError_t launch_gram(const T *Y, int n, int p, T *S, hipStream_t stream)
{
    const int nt = (p + TILE - 1) / TILE;
    const int tiles = nt * (nt + 1) / 2;
    hipLaunchKernelGGL((atb_mfma_kernel<T, true>), dim3(tiles), dim3(256), 0, stream, Y, Y, n,
                       p, p, T(1) / T(n), S);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_atb(const T *A, const T *B, int K, int M, int N, T *C, hipStream_t stream)
{
    dim3 grid((N + TILE - 1) / TILE, (M + TILE - 1) / TILE);
    hipLaunchKernelGGL((atb_mfma_kernel<T, false>), grid, dim3(256), 0, stream, A, B, K, M, N,
                       T(1), C);
    return hipGetLastError();
}

template hipError_t launch_gram<float>(const float *, int, int, float *, hipStream_t);
template hipError_t launch_gram<double>(const double *, int, int, double *, hipStream_t);
template hipError_t launch_atb<float>(const float *, const float *, int, int, int, float *,
                                      hipStream_t);
template hipError_t launch_atb<double>(const double *, const double *, int, int, int, double *,
                                       hipStream_t);

}  // namespace concord
