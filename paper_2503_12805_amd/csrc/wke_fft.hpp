// Register/LDS mixed-radix FFT building blocks for gfx950.
//
// A length-N transform is carried by TPT = N / R_last cooperating lanes;
// lane t holds the V = R_last values x[t + TPT*m], m = 0..V-1, both before
// and after the transform (natural order, no bit reversal).  Stages are
// Stockham autosort steps: the first runs on registers and writes LDS, the
// middle ones run LDS to LDS in place, the last reads LDS into registers.
// Twiddles of the small register DFTs are compile-time constants; the
// inter-stage twiddles come from an N-entry table e^{+2 pi i k / N} that the
// caller keeps in LDS.
//
// DIR = -1 is the forward kernel e^{-2 pi i jk/N}, DIR = +1 the inverse
// (unnormalised).
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <utility>

#include "wke_shape.hpp"

namespace wke {

template <class T> struct cx { T x, y; };

template <class T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.x, s * a.y}; }
template <class T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }

// ---------------------------------------------------------------------------
// Compile-time trigonometry for the register-DFT twiddles: sin and cos of
// 2 pi n / d, reduced exactly to [0, pi/4] and summed as Taylor series
// (enough terms for double rounding on that interval).
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
    double term = x, sum = x;
    for (int k = 1; k < 14; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 14; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
// cos(2 pi n / d) and sin(2 pi n / d) for integers n, d > 0.
struct cs_pair { double c, s; };
constexpr cs_pair cossin2pi(long n, long d) {
    n %= d;
    if (n < 0) n += d;
    // angle = 2 pi n / d = quadrant * pi/2 + phi, phi = pi * rem / (2 d)
    long quad = (4 * n) / d;
    long rem = 4 * n - quad * d;          // phi = pi rem / (2d), rem in [0, d)
    double c0 = 0.0, s0 = 0.0;
    if (2 * rem <= d) {                   // phi <= pi/4
        double phi = kPi * (double)rem / (2.0 * (double)d);
        c0 = taylor_cos(phi);
        s0 = taylor_sin(phi);
    } else {                              // use pi/2 - phi
        double psi = kPi * (double)(d - rem) / (2.0 * (double)d);
        c0 = taylor_sin(psi);
        s0 = taylor_cos(psi);
    }
    switch (quad & 3) {
        case 0: return {c0, s0};
        case 1: return {-s0, c0};
        case 2: return {-c0, -s0};
        default: return {s0, -c0};
    }
}

// multiply by DIR * i (exact)
template <int DIR, class T> __device__ __forceinline__ cx<T> mul_i(cx<T> v) {
    if constexpr (DIR > 0) return {-v.y, v.x};
    else return {v.y, -v.x};
}

// v * e^{DIR 2 pi i NUM / DEN}, with the exact cases folded.
template <int DIR, long NUM, long DEN, class T> __device__ __forceinline__ cx<T> twc(cx<T> v) {
    constexpr long n = ((NUM % DEN) + DEN) % DEN;
    if constexpr (n == 0) {
        return v;
    } else if constexpr (4 * n == DEN) {
        return mul_i<DIR>(v);
    } else if constexpr (2 * n == DEN) {
        return {-v.x, -v.y};
    } else if constexpr (4 * n == 3 * DEN) {
        return mul_i<-DIR>(v);
    } else {
        constexpr cs_pair w = cossin2pi(n, DEN);
        constexpr double c = w.c;
        constexpr double s = DIR > 0 ? w.s : -w.s;
        const T cc = (T)c, ss = (T)s;
        return {cc * v.x - ss * v.y, cc * v.y + ss * v.x};
    }
}

// Barrier between the LDS phases of a transform.  When every lane of a
// transform sits in one wavefront (WAVE), ordering the wave's own LDS
// accesses is enough: LDS instructions of a wave complete in order, so a
// wave-scope fence plus a scheduling barrier replaces the workgroup barrier.
template <bool WAVE> __device__ __forceinline__ void phase_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <int B, int E, class F> __device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int smallest_factor(int n) {
    if (n % 4 == 0 && n != 8 && n != 16) return 4;   // prefer radix-4 splits
    for (int p = 2; p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}
constexpr int split_of(int n) {
    // factor used to split an n-point register DFT: 8 = 2*4, 16 = 4*4,
    // 12 = 4*3, 24 = 4*6 ...
    if (n == 8) return 2;
    if (n == 16) return 4;
    return smallest_factor(n);
}

// In-register n-point DFT (DIR = -1 forward, +1 inverse, unnormalised).
template <int R, int DIR, class T> __device__ __forceinline__ void dft(cx<T>* v);

template <int R, int DIR, class T> struct DftImpl {
    __device__ __forceinline__ static void run(cx<T>* v) {
        // R = P * Q: input n = Q*n1 + n2, output k = k1 + P*k2
        constexpr int P = split_of(R);
        constexpr int Q = R / P;
        cx<T> tmp[R];
        static_for<0, Q>([&](auto n2c) {
            constexpr int n2 = decltype(n2c)::value;
            cx<T> u[P];
            static_for<0, P>([&](auto n1c) {
                constexpr int n1 = decltype(n1c)::value;
                u[n1] = v[Q * n1 + n2];
            });
            dft<P, DIR>(u);
            static_for<0, P>([&](auto k1c) {
                constexpr int k1 = decltype(k1c)::value;
                tmp[n2 * P + k1] = twc<DIR, (long)n2 * k1, R>(u[k1]);
            });
        });
        static_for<0, P>([&](auto k1c) {
            constexpr int k1 = decltype(k1c)::value;
            cx<T> z[Q];
            static_for<0, Q>([&](auto n2c) {
                constexpr int n2 = decltype(n2c)::value;
                z[n2] = tmp[n2 * P + k1];
            });
            dft<Q, DIR>(z);
            static_for<0, Q>([&](auto k2c) {
                constexpr int k2 = decltype(k2c)::value;
                v[k1 + P * k2] = z[k2];
            });
        });
    }
};

template <int DIR, class T> struct DftImpl<1, DIR, T> {
    __device__ __forceinline__ static void run(cx<T>*) {}
};
template <int DIR, class T> struct DftImpl<2, DIR, T> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};
template <int DIR, class T> struct DftImpl<3, DIR, T> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        const T half = (T)0.5;
        const T s3 = (T)0.86602540378443864676372317075293618;   // sin(2 pi / 3)
        cx<T> t1 = v[1] + v[2];
        cx<T> t2 = v[0] - half * t1;
        cx<T> d = v[1] - v[2];
        cx<T> rot = mul_i<DIR>(d);       // DIR i (v1 - v2)
        v[0] = v[0] + t1;
        v[1] = t2 + s3 * rot;
        v[2] = t2 - s3 * rot;
    }
};
template <int DIR, class T> struct DftImpl<4, DIR, T> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        cx<T> a = v[0] + v[2], b = v[0] - v[2];
        cx<T> c = v[1] + v[3], d = mul_i<DIR>(v[1] - v[3]);
        v[0] = a + c;
        v[2] = a - c;
        v[1] = b + d;
        v[3] = b - d;
    }
};

template <int R, int DIR, class T> __device__ __forceinline__ void dft(cx<T>* v) { DftImpl<R, DIR, T>::run(v); }

// Scratch layout of a transform.  Unpadded (PAD = 0), element e sits at
// s[e * stride] (a strided view, e.g. a column of an LDS plane, or one of
// several transforms interleaved element by element).  Padded, one spare
// slot follows every PAD elements, s[(e + e / PAD) * stride]: the first
// stage writes runs of R0 consecutive elements per lane, i.e. lanes R0
// elements apart, which without padding fall on the same LDS banks.
// (e >= 0: the division is unsigned, a shift for the power-of-two steps)
template <int PAD> __device__ __forceinline__ int sidx(int e) {
    return PAD ? e + (int)((unsigned)e / (unsigned)PAD) : e;
}

// Middle stages (radix list without the first and the last entry).
template <class T, int N, int DIR, bool WAVE, int PAD, int NS, int... Rs> struct MidStages;
template <class T, int N, int DIR, bool WAVE, int PAD, int NS> struct MidStages<T, N, DIR, WAVE, PAD, NS> {
    static constexpr int ns_out = NS;
    __device__ __forceinline__ static void run(cx<T>*, int, int, const cx<T>*, bool) {}
};
template <class T, int N, int DIR, bool WAVE, int PAD, int NS, int R, int... Rs>
struct MidStages<T, N, DIR, WAVE, PAD, NS, R, Rs...> {
    static constexpr int ns_out = MidStages<T, N, DIR, WAVE, PAD, NS * R, Rs...>::ns_out;
    __device__ __forceinline__ static void run(cx<T>* s, int stride, int t, const cx<T>* tw, bool active) {
        constexpr int TPT = FftShape<N>::TPT;
        constexpr int nb = N / R;
        constexpr int per = (nb + TPT - 1) / TPT;
        cx<T> u[per][R];
        phase_sync<WAVE>();
        if (active) {
#pragma unroll
            for (int k = 0; k < per; ++k) {
                const int i = t + TPT * k;
                if (i < nb) {
                    const int j = i % NS;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        cx<T> w = tw[r * j * (N / (NS * R))];
                        if (DIR < 0) w = conj(w);
                        u[k][r] = s[sidx<PAD>(i + r * nb) * stride] * w;
                    }
                }
            }
        }
        phase_sync<WAVE>();
        if (active) {
#pragma unroll
            for (int k = 0; k < per; ++k) {
                const int i = t + TPT * k;
                if (i < nb) {
                    const int j = i % NS;
                    dft<R, DIR>(u[k]);
#pragma unroll
                    for (int r = 0; r < R; ++r) s[sidx<PAD>((i / NS) * NS * R + j + r * NS) * stride] = u[k][r];
                }
            }
        }
        MidStages<T, N, DIR, WAVE, PAD, NS * R, Rs...>::run(s, stride, t, tw, active);
    }
};

template <class T, int N, int DIR, bool WAVE, int PAD, class P> struct MidOf;
template <class T, int N, int DIR, bool WAVE, int PAD, int R0, int... Rs>
struct MidOf<T, N, DIR, WAVE, PAD, Radices<R0, Rs...>> {
    // drop the last radix from Rs...
    template <int... A> struct Drop;
    template <int A0> struct Drop<A0> { using mid = MidStages<T, N, DIR, WAVE, PAD, R0>; };
    template <int A0, int A1> struct Drop<A0, A1> { using mid = MidStages<T, N, DIR, WAVE, PAD, R0, A0>; };
    template <int A0, int A1, int A2> struct Drop<A0, A1, A2> { using mid = MidStages<T, N, DIR, WAVE, PAD, R0, A0, A1>; };
    using type = typename Drop<Rs...>::mid;
};

// The distributed transform.  All lanes of the workgroup (of the wavefront
// when WAVE) must call it together (it contains barriers when NST > 1);
// lanes with active == false take part in the barriers only.  s points at
// this transform's LDS slots (element e at s[e * stride], or, when PAD > 0,
// at s[(e + e / PAD) * stride], N + (N - 1) / PAD slots); tw is the
// N-entry table e^{+2 pi i k/N} in LDS, written before the first call and
// ordered by a workgroup barrier.
template <class T, int N, int DIR, bool WAVE = false, int PAD = 0>
__device__ __forceinline__ void fft_dist(cx<T>* v, cx<T>* s, int stride, int t, const cx<T>* tw, bool active) {
    using S = FftShape<N>;
    constexpr int R0 = S::R0, RL = S::RL, TPT = S::TPT;
    if constexpr (S::NST == 1) {
        if (active) dft<N, DIR>(v);
    } else {
        phase_sync<WAVE>();   // earlier readers of s are done
        if (active) {
            constexpr int nb0 = N / R0;
            constexpr int per0 = RL / R0;
#pragma unroll
            for (int k = 0; k < per0; ++k) {
                const int i = t + TPT * k;
                cx<T> u[R0];
#pragma unroll
                for (int r = 0; r < R0; ++r) u[r] = v[k + r * (nb0 / TPT)];
                dft<R0, DIR>(u);
#pragma unroll
                for (int r = 0; r < R0; ++r) s[sidx<PAD>(i * R0 + r) * stride] = u[r];
            }
        }
        using Mid = typename MidOf<T, N, DIR, WAVE, PAD, typename S::P>::type;
        Mid::run(s, stride, t, tw, active);
        static_assert(Mid::ns_out == TPT, "stage spans must multiply to N / R_last");
        phase_sync<WAVE>();
        if (active) {
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                cx<T> w = tw[r * t];
                if (DIR < 0) w = conj(w);
                v[r] = s[sidx<PAD>(t + r * TPT) * stride] * w;
            }
            dft<RL, DIR>(v);
        }
    }
}

}  // namespace wke
