// Closed form of the circle-method round-robin table (Section 3.2, Algorithm 1).
//
// Vertex 0 is the fixed position of the table; vertices 1..p_even-1 sit on a
// circle of m = p_even - 1 positions, circle coordinate x = v - 1.  After r
// rotations the circle entry at table position s (2 <= s <= p_even, 1-based)
// is ((s - 2 - r) mod m) + 1, so
//   slot 0      pairs vertex 0 with circle x = (m - 1 - r) mod m,
//   slot q >= 1 pairs circle x_a = (q - 1 - r) mod m with x_b = (m - 1 - q - r) mod m.
// Hence two circle vertices x != y share colour r iff x + y = -2 (r + 1) (mod m),
// and the circle vertex with 2x = -2 (r + 1) is the one paired with vertex 0.
// For odd p the vertex p (the paper's dummy p + 1) idles its partner.
//
// Everything is plain int32 arithmetic, usable on host and device; nothing is
// tabulated (a table would hold p^2 entries).
#pragma once

#include <hip/hip_runtime.h>

namespace concord {

struct Circle {
    int p;   // vertices
    int pe;  // p_even
    int m;   // colours = pe - 1
    int H;   // slots per colour = pe / 2

    __host__ __device__ static Circle make(int p_)
    {
        Circle c;
        c.p = p_;
        c.pe = p_ + (p_ & 1);
        c.m = c.pe - 1;
        c.H = c.pe / 2;
        return c;
    }

    // 0 <= a < 4m is all this is ever called with.
    __host__ __device__ int mod(int a) const { return a % m; }

    // Partner of vertex v (0 <= v < p) in colour r, or -1 when v idles
    // (its partner is the dummy vertex of odd p).
    __host__ __device__ int partner(int r, int v) const
    {
        int w;
        if (v == 0) {
            w = mod(2 * m - 1 - r) + 1;
        } else {
            int x = v - 1;
            int y = mod(4 * m - 2 * (r + 1) - x);
            w = (y == x) ? 0 : y + 1;
        }
        return (w >= p) ? -1 : w;
    }

    // Slot of vertex v in colour r (the slot of the pair holding v).
    __host__ __device__ int slot(int r, int v) const
    {
        if (v == 0)
            return 0;
        int q = mod(v + r);  // (x + 1 + r) mod m with x = v - 1
        if (q == 0)
            return 0;
        return q < H ? q : m - q;
    }

    // The pair in slot q of colour r: (a, b) in table order (either may equal
    // p for odd p, the dummy).
    __host__ __device__ void pair(int r, int q, int *a, int *b) const
    {
        if (q == 0) {
            *a = 0;
            *b = mod(2 * m - 1 - r) + 1;
        } else {
            *a = mod(2 * m + q - 1 - r) + 1;
            *b = mod(3 * m - 1 - q - r) + 1;
        }
    }

    // Colour of the edge {u, v}, u != v.  2 is invertible mod the odd m,
    // with inverse H = (m + 1) / 2.
    __host__ __device__ int colour(int u, int v) const
    {
        if (u > v) {
            int t = u;
            u = v;
            v = t;
        }
        if (u == 0)
            return mod(2 * m - 1 - (v - 1));
        long long s = (long long)(u - 1) + (v - 1);  // x + y
        // r + 1 = -(x + y) * H (mod m)
        long long rp1 = ((-(s % m) + m) % m) * (long long)H % m;
        return (int)((rp1 - 1 + m) % m);
    }
};

}  // namespace concord
