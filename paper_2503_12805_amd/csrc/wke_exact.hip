// Exact-weight reference system (Appendix B): the Galerkin sums of eqs.
// (KK1)-(KK4) with the exact constraint l + m + n = j and the weight
// functions integrated in closed form over q-hat and sigma.  With the sphere
// mean S(x) = int e^{i x.s} ds (2 pi J_0(x) on the circle, 4 pi sin(x)/x on
// the sphere) each weight is
//   Phi(a, b) = int_0^R r^(2d-3) S(pi r sqrt(a) / (2L)) S(pi r sqrt(b) / (2L)) dr
// of two squared integer norms: G_1 = Phi(|2m+l+n|^2, |l-n|^2),
// G_2 = Phi(|2m+n|^2, |n|^2), G_3 = Phi(|l+n|^2, |l-n|^2), G_4 = Phi(|2m+l|^2, |l|^2).
// The radial integral is Gauss-Legendre; Phi is then a small dense product
// S diag(u) S^T, built once per call.  The sum over (l, m) is O(N^(3d)):
// tiny N only.
#include <hip/hip_runtime.h>

#include <mutex>

#include "wke_internal.hpp"

namespace wke {

// Workspace of the allocation-free variant (wke_exact_system_noalloc): a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes its name to a kernel (on the host the name is only a
// stand-in for the symbol): it uses the device address looked up below.
static __device__ __align__(256) double scratch[EXACT_SCRATCH_DOUBLES];

hipError_t exact_scratch(double** ptr) {
    static std::mutex mu;
    static double* addr[EXACT_MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= EXACT_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // once per device, with that device current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double*>(p);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

namespace {

__device__ __forceinline__ int signed_mode(int i, int N) { return i < N / 2 ? i : i - N; }

__global__ void k_ex_nodes(ExactArgs a) {
    for (int i = threadIdx.x; i < a.nr; i += blockDim.x) {
        double x, w;
        gl_root(a.nr, i, &x, &w);
        const double r = 0.5 * a.R * (1.0 + x);
        double rp = 1.0;
        for (int k = 0; k < 2 * a.d - 3; ++k) rp *= r;
        a.rk[i] = r;
        a.uk[i] = 0.5 * a.R * w * rp;
    }
}

// S[a][k] = S(pi r_k sqrt(a) / (2L))
__global__ void k_ex_sphere(ExactArgs a) {
    const long long total = (long long)(a.A + 1) * a.nr;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int q = (int)(e / a.nr), k = (int)(e % a.nr);
        const double x = M_PI * a.rk[k] * sqrt((double)q) / (2.0 * a.L);
        a.S[e] = a.d == 2 ? 2.0 * M_PI * j0(x) : (x == 0.0 ? 4.0 * M_PI : 4.0 * M_PI * sin(x) / x);
    }
}

// Phi = S[0..A] diag(u) S[0..B]^T, 16 x 16 output tiles, 16-wide chunks of
// the radial index staged in LDS.
__global__ __launch_bounds__(256) void k_ex_phi(ExactArgs a) {
    __shared__ double sa[16][17], sb[16][17];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;   // a, b
    double acc = 0.0;
    for (int k0 = 0; k0 < a.nr; k0 += 16) {
        const int ka = k0 + tx;
        const int ra = blockIdx.y * 16 + ty, cb = blockIdx.x * 16 + ty;
        sa[ty][tx] = (ra <= a.A && ka < a.nr) ? a.S[(long long)ra * a.nr + ka] * a.uk[ka] : 0.0;
        sb[ty][tx] = (cb <= a.B && ka < a.nr) ? a.S[(long long)cb * a.nr + ka] : 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) acc += sa[ty][k] * sb[tx][k];
        __syncthreads();
    }
    if (row <= a.A && col <= a.B) a.phi[(long long)row * (a.B + 1) + col] = acc;
}

// Direct transforms with the grid offset k_x = -L + h x folded in:
// dir -1: F_j = N^-d (-1)^(sum j) sum_x f(x) e^{-2 pi i j.x / N};
// dir +1: Q(x) = sum_j (-1)^(sum j) Qh_j e^{+2 pi i j.x / N}.
__global__ void k_ex_dft(int d, int N, int dir, const double2* in, double2* out) {
    long long n = 1;
    for (int k = 0; k < d; ++k) n *= N;
    const long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (o >= n) return;
    int oi[3] = {0, 0, 0};
    long long rem = o;
    for (int k = d - 1; k >= 0; --k) { oi[k] = (int)(rem % N); rem /= N; }
    double sx = 0.0, sy = 0.0;
    for (long long p = 0; p < n; ++p) {
        int pi_[3] = {0, 0, 0};
        long long r2 = p;
        for (int k = d - 1; k >= 0; --k) { pi_[k] = (int)(r2 % N); r2 /= N; }
        // mode index j and grid index x, whichever side is which
        const int* jx = dir < 0 ? oi : pi_;
        const int* xx = dir < 0 ? pi_ : oi;
        long long ph = 0;
        int sgn = 0;
        for (int k = 0; k < d; ++k) {
            const int j = signed_mode(jx[k], N);
            ph += (long long)(((j % N) + N) % N) * xx[k];
            sgn += j;
        }
        double sn, cs;
        sincospi(2.0 * (double)(ph % N) / N, &sn, &cs);
        if (dir < 0) sn = -sn;
        if (sgn & 1) { cs = -cs; sn = -sn; }
        const double2 v = in[p];
        sx += v.x * cs - v.y * sn;
        sy += v.x * sn + v.y * cs;
    }
    const double sc = dir < 0 ? 1.0 / (double)n : 1.0;
    out[o] = make_double2(sc * sx, sc * sy);
}

// Q hat of one mode j per workgroup: its lanes split the (l, m) pairs, then a
// fixed-order tree sum in LDS.
__global__ __launch_bounds__(256) void k_ex_sum(ExactArgs a) {
    __shared__ double2 Fs[1024];
    __shared__ double2 red[256];
    const int d = a.d, N = a.N;
    int n = 1;
    for (int k = 0; k < d; ++k) n *= N;
    const double2* F = reinterpret_cast<const double2*>(a.F);
    for (int i = threadIdx.x; i < n; i += 256) Fs[i] = F[i];
    __syncthreads();
    int jv[3] = {0, 0, 0};
    {
        int rem = blockIdx.x;
        for (int k = d - 1; k >= 0; --k) { jv[k] = signed_mode(rem % N, N); rem /= N; }
    }
    const long long B1 = a.B + 1;
    double sx = 0.0, sy = 0.0;
    for (long long p = threadIdx.x; p < (long long)n * n; p += 256) {
        int li = (int)(p / n), mi = (int)(p % n);
        int l[3] = {0, 0, 0}, m[3] = {0, 0, 0}, v[3] = {0, 0, 0};
        for (int k = d - 1; k >= 0; --k) {
            l[k] = signed_mode(li % N, N);
            li /= N;
            m[k] = signed_mode(mi % N, N);
            mi /= N;
        }
        bool ok = true;
        int vi = 0;
        int q1 = 0, q2 = 0, q3 = 0, q4 = 0, q5 = 0, q7 = 0, q8 = 0;
        for (int k = 0; k < d; ++k) {
            v[k] = jv[k] - l[k] - m[k];
            if (v[k] < -N / 2 || v[k] > N / 2 - 1) ok = false;
            vi = vi * N + (v[k] < 0 ? v[k] + N : v[k]);
            const int u1 = 2 * m[k] + l[k] + v[k], u2 = l[k] - v[k], u3 = 2 * m[k] + v[k];
            const int u4 = l[k] + v[k], u5 = 2 * m[k] + l[k];
            q1 += u1 * u1;
            q2 += u2 * u2;
            q3 += u3 * u3;
            q4 += v[k] * v[k];
            q5 += u4 * u4;
            q7 += u5 * u5;
            q8 += l[k] * l[k];
        }
        if (!ok) continue;
        const double G = a.phi[q1 * B1 + q2] - a.phi[q3 * B1 + q4] + a.phi[q5 * B1 + q2] - a.phi[q7 * B1 + q8];
        const double2 fl = Fs[p / n], fm = Fs[p % n], fv = Fs[vi];
        const double px = fl.x * fm.x - fl.y * fm.y, py = fl.x * fm.y + fl.y * fm.x;
        sx += G * (px * fv.x - py * fv.y);
        sy += G * (px * fv.y + py * fv.x);
    }
    red[threadIdx.x] = make_double2(sx, sy);
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[threadIdx.x].x += red[threadIdx.x + h].x;
            red[threadIdx.x].y += red[threadIdx.x + h].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double qs = ldexp(1.0, 1 - d);
        reinterpret_cast<double2*>(a.Qh)[blockIdx.x] = make_double2(qs * red[0].x, qs * red[0].y);
    }
}

}  // namespace

hipError_t launch_exact(const ExactArgs& a, hipStream_t s) {
    int n = 1;
    for (int k = 0; k < a.d; ++k) n *= a.N;
    if (n > 1024 || a.nr < 1 || a.A < 0 || a.B < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ex_nodes, dim3(1), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long ns = (long long)(a.A + 1) * a.nr;
    hipLaunchKernelGGL(k_ex_sphere, dim3((unsigned)((ns + 255) / 256 > 65535 ? 65535 : (ns + 255) / 256)), dim3(256), 0,
                       s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ex_phi, dim3((a.B + 16) / 16, (a.A + 16) / 16), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ex_dft, dim3((n + 255) / 256), dim3(256), 0, s, a.d, a.N, -1,
                       reinterpret_cast<const double2*>(a.f), reinterpret_cast<double2*>(a.F));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ex_sum, dim3(n), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ex_dft, dim3((n + 255) / 256), dim3(256), 0, s, a.d, a.N, 1,
                       reinterpret_cast<const double2*>(a.Qh), reinterpret_cast<double2*>(a.Q));
    return hipGetLastError();
}

}  // namespace wke
