// Register/LDS 2D FFT of the persistent kernels: one workgroup holds an
// N x N complex field (N = 8 P, P in {4, 8, 16}), 16 values per thread
// (N^2/16 threads).  A 2D FFT is four passes, radix-8 and radix-P along each
// dimension:
//   rows    x = x0 + P m,  kx = k1 + 8 k2   (pass A: radix-8 over m,  pass B: radix-P over x0)
//   columns y = y0 + 8 m,  ky = k1 + P k2   (pass C: radix-P over m,  pass D: radix-8 over y0)
// with twiddles W_N^(x0 k1) after A and W_N^(y0 k1) after C.  The forward
// transform runs A, B, C, D (decimation in frequency); the inverse runs the
// transposed passes D', C', B', A' (decimation in time), so the Fourier-space
// update happens in pass D's registers and the pixel-space update in pass A's,
// and LDS is touched only for the three exchanges between passes.
//
// LDS exchanges place each row at a base of its own and keep the column in
// order, so that the elements one thread moves in an exchange lie at constant
// offsets from one base (the immediate offsets of ds_read/ds_write, no address
// arithmetic per element), while every 16- or 32-lane phase of an LDS
// instruction still touches distinct banks:
//   E1  row y starts at y N + 2 s(y) + 32 (y / R1), s(y) = (P/2)(y % R1) + (y / R1) % (P/2):
//       the R1 rows of one 16-lane phase of pass A's 16-byte accesses fall
//       on disjoint 128-byte halves of the banks, and 16 consecutive rows
//       (pass B's lanes) on 16 distinct 16-byte bank groups;
//   E2  pitch N + 1 (pass B's lanes walk rows, pass C's walk columns);
//   E3  pitch N + 1 as well (both sides' lanes walk columns).
// Four of a sweep's twelve block barriers are not needed: in the exchanges
// C -> C (E2 read, E3 written, and back), D -> D and A -> A each thread writes
// exactly the addresses it has just read (E2 and E3 share a layout), and a
// wave's LDS operations take effect in order, so no other thread can still be
// waiting for what it overwrites.  A caller that writes LDS between two
// transforms synchronises the block first.
// Twiddles W_N^(a b) sit in LDS in one small table per pass, row a (the
// thread's own index: x0 in A, k1 in B and D, y0 in C) by column b (the
// register's), so that a thread's twiddles too lie at constant offsets from
// one base.  Pass A's rows have pitch 9, so that the eight rows one wave reads
// fall on distinct banks; the other passes read one or a few rows per wave.
#pragma once
#include "mf_device.hpp"

namespace mf {

namespace {

template <int N>
struct Res {
    static constexpr int P = N / 8;
    static constexpr int NT = N * N / 16;                  // threads per workgroup
    static constexpr int TB = 16 / P;                      // radix-P tasks per thread
    static constexpr int R1 = 32 / P;                      // pass-A rows per 16-lane phase
    static constexpr int LDS = N * N + N * P;              // float2 elements of the exchange buffer (E1's extent)
    // twiddle tables: A [x0 < P][k1 < 8] pitch 9, B [k1 < 8][x0 < P],
    // C [y0 < 8][k1 < P], D [k1 < P][y0 < 8]
    static constexpr int TWA = 0, TWB = TWA + 9 * P, TWC = TWB + 8 * P, TWD = TWC + 8 * P;
    static constexpr int TWS = TWD + 8 * P;                // float2 elements of the four tables
};

// Fill the twiddle tables from W_N^r (r < N); every product a b is below N.
// Visible to the block after its next barrier.
template <int N>
__device__ __forceinline__ void fill_twiddle_tables(float2* t, const float2* __restrict__ tw, unsigned tid) {
    constexpr int P = Res<N>::P;
    for (unsigned e = tid; e < (unsigned)Res<N>::TWS; e += Res<N>::NT) {
        unsigned r;
        if (e < (unsigned)Res<N>::TWB) {
            const unsigned q = e - Res<N>::TWA, a = q / 9, b = q % 9;
            r = b < 8 ? a * b : 0;
        } else if (e < (unsigned)Res<N>::TWC) {
            const unsigned q = e - Res<N>::TWB;
            r = (q / P) * (q % P);
        } else if (e < (unsigned)Res<N>::TWD) {
            const unsigned q = e - Res<N>::TWC;
            r = (q / P) * (q % P);
        } else {
            const unsigned q = e - Res<N>::TWD;
            r = (q / 8) * (q % 8);
        }
        t[e] = tw[r];
    }
}

// E1 (between passes A and B): row y, column k1 P + x0
template <int N>
__device__ __forceinline__ unsigned e1_row(unsigned r) {
    constexpr unsigned P = Res<N>::P, R1 = Res<N>::R1;
    return r * N + 2 * ((P / 2) * (r % R1) + (r / R1) % (P / 2)) + 32 * (r / R1);
}
template <int N>
__device__ __forceinline__ unsigned e1(unsigned r, unsigned c) {
    return e1_row<N>(r) + c;
}
// E2 (between passes B and C): row y, column kx
template <int N>
__device__ __forceinline__ unsigned e2(unsigned r, unsigned c) {
    return r * (N + 1) + c;
}
// E3 (between passes C and D): row 8 k1 + y0, column kx
template <int N>
__device__ __forceinline__ unsigned e3(unsigned r, unsigned c) {
    return r * (N + 1) + c;
}

__device__ __forceinline__ void st2(float2* lds, unsigned i, float2 a, float2 b) {
    *reinterpret_cast<float4*>(lds + i) = make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ void ld2(const float2* lds, unsigned i, float2& a, float2& b) {
    const float4 q = *reinterpret_cast<const float4*>(lds + i);
    a = make_float2(q.x, q.y);
    b = make_float2(q.z, q.w);
}

template <int R, bool INV>
__device__ __forceinline__ void dft_slice(float2* v) {
    float2 t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[i] = v[i];
    dft<R, INV>(t);
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[i];
}

// Hide a pointer from loop-invariant code motion: tables are re-read (from
// cache) every sweep instead of being held in registers across sweeps.
// An opaque zero, to offset an LDS table per sweep without losing its address space.
__device__ __forceinline__ unsigned per_sweep_zero() {
    unsigned z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

template <typename T>
__device__ __forceinline__ const T* per_sweep(const T* p) {
    // an opaque zero offset (not the pointer itself), so that the pointer
    // keeps its global address space: flat loads would also count against
    // the LDS wait counter
    unsigned z = 0;
    asm volatile("" : "+s"(z));
    return p + z;
}

template <bool INV>
__device__ __forceinline__ float2 twiddle(float2 v, const float2* __restrict__ row, int col) {
    const float2 w = row[col];
    return INV ? cmulc(v, w) : cmul(v, w);
}

// ---------------------------------------------------------------- passes --
// Thread coordinates in each layout (tid in [0, NT)):
//   A: y = tid / (P/2), j = tid % (P/2); holds x = 2j + q + P m     at v[8q + m]
//   B: t = tid + i NT (i < TB): y = t % N, k1 = t / N; holds x0    at v[P i + x0]
//   C: kx = tid % N, y0 = tid / N + i P/2 (i < TB);   holds m      at v[P i + m]
//   D: jx = tid % (N/2), k1 = tid / (N/2); kx = 2jx + q; holds y0  at v[8q + y0]

template <int N, bool INV>
__device__ __forceinline__ void pass_A(float2 (&v)[16], const float2* __restrict__ tw, unsigned tid) {
    constexpr int P = Res<N>::P;
    const unsigned j = tid % (P / 2);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        dft_slice<8, INV>(v + 8 * q);
        if (!INV) {
            const float2* row = tw + Res<N>::TWA + 9 * (2 * j + q);
#pragma unroll
            for (int k1 = 1; k1 < 8; ++k1) v[8 * q + k1] = twiddle<false>(v[8 * q + k1], row, k1);
        }
    }
}

template <int N>
__device__ __forceinline__ void store_E1_from_A(float2* lds, const float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P;
    const unsigned y = tid / (P / 2), j = tid % (P / 2);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) st2(lds, e1<N>(y, k1 * P + 2 * j), v[k1], v[8 + k1]);
}

template <int N>
__device__ __forceinline__ void load_A_from_E1(const float2* lds, float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P;
    const unsigned y = tid / (P / 2), j = tid % (P / 2);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) ld2(lds, e1<N>(y, k1 * P + 2 * j), v[k1], v[8 + k1]);
}

template <int N>
__device__ __forceinline__ void load_B_from_E1(const float2* lds, float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned t = tid + i * NT, y = t % N, k1 = t / N;
#pragma unroll
        for (int x0 = 0; x0 < P; x0 += 2) ld2(lds, e1<N>(y, k1 * P + x0), v[P * i + x0], v[P * i + x0 + 1]);
    }
}

template <int N>
__device__ __forceinline__ void store_E1_from_B(float2* lds, const float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned t = tid + i * NT, y = t % N, k1 = t / N;
#pragma unroll
        for (int x0 = 0; x0 < P; x0 += 2) st2(lds, e1<N>(y, k1 * P + x0), v[P * i + x0], v[P * i + x0 + 1]);
    }
}

// pass B: forward radix-P over x0 -> k2 (no twiddle after);
// inverse: radix-P over k2 -> x0, then twiddle conj W_N^(x0 k1).
template <int N, bool INV>
__device__ __forceinline__ void pass_B(float2 (&v)[16], const float2* __restrict__ tw, unsigned tid) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        dft_slice<P, INV>(v + P * i);
        if (INV) {
            const float2* row = tw + Res<N>::TWB + P * ((tid + i * NT) / N);
#pragma unroll
            for (int x0 = 1; x0 < P; ++x0) v[P * i + x0] = twiddle<true>(v[P * i + x0], row, x0);
        }
    }
}

template <int N>
__device__ __forceinline__ void store_E2_from_B(float2* lds, const float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned t = tid + i * NT, y = t % N, k1 = t / N;
#pragma unroll
        for (int k2 = 0; k2 < P; ++k2) lds[e2<N>(y, k1 + 8 * k2)] = v[P * i + k2];
    }
}

template <int N>
__device__ __forceinline__ void load_B_from_E2(const float2* lds, float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned t = tid + i * NT, y = t % N, k1 = t / N;
#pragma unroll
        for (int k2 = 0; k2 < P; ++k2) v[P * i + k2] = lds[e2<N>(y, k1 + 8 * k2)];
    }
}

template <int N>
__device__ __forceinline__ void load_C_from_E2(const float2* lds, float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
    const unsigned kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int m = 0; m < P; ++m) v[P * i + m] = lds[e2<N>(y0 + 8 * m, kx)];
    }
}

template <int N>
__device__ __forceinline__ void store_E2_from_C(float2* lds, const float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
    const unsigned kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int m = 0; m < P; ++m) lds[e2<N>(y0 + 8 * m, kx)] = v[P * i + m];
    }
}

// pass C: forward radix-P over m -> k1, then twiddle W_N^(y0 k1);
// inverse: radix-P over k1 -> m (the twiddle was applied in D').
template <int N, bool INV>
__device__ __forceinline__ void pass_C(float2 (&v)[16], const float2* __restrict__ tw, unsigned tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        dft_slice<P, INV>(v + P * i);
        if (!INV) {
            const float2* row = tw + Res<N>::TWC + P * (tid / N + i * (P / 2));
#pragma unroll
            for (int k1 = 1; k1 < P; ++k1) v[P * i + k1] = twiddle<false>(v[P * i + k1], row, k1);
        }
    }
}

template <int N>
__device__ __forceinline__ void store_E3_from_C(float2* lds, const float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
    const unsigned kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) lds[e3<N>(k1 * 8 + y0, kx)] = v[P * i + k1];
    }
}

template <int N>
__device__ __forceinline__ void load_C_from_E3(const float2* lds, float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
    const unsigned kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) v[P * i + k1] = lds[e3<N>(k1 * 8 + y0, kx)];
    }
}

// (8-byte accesses: at pitch N + 1 a pair of columns is not 16-byte aligned)
template <int N>
__device__ __forceinline__ void load_D_from_E3(const float2* lds, float2 (&v)[16], unsigned tid) {
    const unsigned jx = tid % (N / 2), k1 = tid / (N / 2);
#pragma unroll
    for (int y0 = 0; y0 < 8; ++y0) {
        const unsigned i = e3<N>(k1 * 8 + y0, 2 * jx);
        v[y0] = lds[i];
        v[8 + y0] = lds[i + 1];
    }
}

template <int N>
__device__ __forceinline__ void store_E3_from_D(float2* lds, const float2 (&v)[16], unsigned tid) {
    const unsigned jx = tid % (N / 2), k1 = tid / (N / 2);
#pragma unroll
    for (int y0 = 0; y0 < 8; ++y0) {
        const unsigned i = e3<N>(k1 * 8 + y0, 2 * jx);
        lds[i] = v[y0];
        lds[i + 1] = v[8 + y0];
    }
}

// pass D: forward radix-8 over y0 -> k2 (ky = k1 + P k2);
// inverse: radix-8 over k2 -> y0, then twiddle conj W_N^(y0 k1).
template <int N, bool INV>
__device__ __forceinline__ void pass_D(float2 (&v)[16], const float2* __restrict__ tw, unsigned tid) {
    const float2* row = tw + Res<N>::TWD + 8 * (tid / (N / 2));
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        dft_slice<8, INV>(v + 8 * q);
        if (INV) {
#pragma unroll
            for (int y0 = 1; y0 < 8; ++y0) v[8 * q + y0] = twiddle<true>(v[8 * q + y0], row, y0);
        }
    }
}

// tw: the four twiddle tables in LDS (fill_twiddle_tables).
template <int N>
__device__ __forceinline__ void forward_fft(float2 (&v)[16], float2* lds, const float2* __restrict__ tw, unsigned tid) {
    pass_A<N, false>(v, tw, tid);
    store_E1_from_A<N>(lds, v, tid);
    __syncthreads();
    load_B_from_E1<N>(lds, v, tid);
    __syncthreads();
    pass_B<N, false>(v, tw, tid);
    store_E2_from_B<N>(lds, v, tid);
    __syncthreads();
    load_C_from_E2<N>(lds, v, tid);
    pass_C<N, false>(v, tw, tid);
    store_E3_from_C<N>(lds, v, tid);  // the addresses this thread read from E2
    __syncthreads();
    load_D_from_E3<N>(lds, v, tid);
    pass_D<N, false>(v, tw, tid);
}

template <int N>
__device__ __forceinline__ void inverse_fft(float2 (&v)[16], float2* lds, const float2* __restrict__ tw, unsigned tid) {
    pass_D<N, true>(v, tw, tid);
    store_E3_from_D<N>(lds, v, tid);
    __syncthreads();
    load_C_from_E3<N>(lds, v, tid);
    pass_C<N, true>(v, tw, tid);
    store_E2_from_C<N>(lds, v, tid);  // the addresses this thread read from E3
    __syncthreads();
    load_B_from_E2<N>(lds, v, tid);
    __syncthreads();
    pass_B<N, true>(v, tw, tid);
    store_E1_from_B<N>(lds, v, tid);
    __syncthreads();
    load_A_from_E1<N>(lds, v, tid);
    pass_A<N, true>(v, tw, tid);
}

}  // namespace

}  // namespace mf
