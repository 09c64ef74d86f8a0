// HIP kernels of the wke library for gfx950 (MI355X).
//
// One evaluation of Q (Alg. 1 of the paper, reorganised for the GPU):
//   colfwd  : spec0 = axis-0 forward DFT of the grid state / N^d
//   passA   : per slab j0 of axis 0, finish the forward transform over the
//             remaining axes (giving f_hat), then for every shifted field s
//             (a per (p1, p2) item, b/c per collision angle) multiply by the
//             separable phase exp(-i pi j.s / L) and inverse-transform the
//             remaining axes; the result is written to G[s][j0][...].
//   passB   : per column of axis 0, inverse-transform every G[s] column
//             (this finishes f_N(k_x - s) on the grid), form the cubic
//             product of Alg. 1 for each quadrature unit and accumulate the
//             weighted sum; epilogue writes Q, or performs the RK4 stage
//             update and the next axis-0 forward transform.
//   fused (2D): the column pass builds the slab fields of its own column
//             directly from spec0 by periodic interpolation along axis 1
//             (a sum over x1 with a per-field kernel), so that one launch
//             per evaluation does all of passA and passB.
// The per-point forward transform of each product in Alg. 1 is dropped:
// it is followed by an inverse transform of the same size, and the sum over
// quadrature points commutes with the (linear) transform, so Q on the grid
// is the weighted sum of the products on the grid.
#include <hip/hip_ext.h>

#include "wke_fft.hpp"
#include "wke_internal.hpp"

namespace wke {

template <class T> struct Tr;
template <> struct Tr<double> { static __device__ __forceinline__ double ab(double v) { return fabs(v); } };
template <> struct Tr<float>  { static __device__ __forceinline__ float ab(float v) { return fabsf(v); } };

// Compensated (Neumaier) accumulation for float; plain for double.
template <class T> __device__ __forceinline__ void acc_add(T& s, T& c, T x) {
    if constexpr (std::is_same<T, float>::value) {
        T t = s + x;
        if (Tr<T>::ab(s) >= Tr<T>::ab(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    } else {
        (void)c;
        s += x;
    }
}

template <class T> __device__ __forceinline__ cx<T> to_t(double2 v) { return {(T)v.x, (T)v.y}; }

// 16 x 16 x 4 matrix-core tile, D += A B.  Lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] and holds four elements of D in column l % 16: rows
// l / 16 + 4 r (double) or 4 (l / 16) + r (float), r = 0..3.
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
template <class T> struct Mfma;
template <> struct Mfma<double> {
    using acc_t = mf_d4;
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return lane / 16 + 4 * r; }
};
template <> struct Mfma<float> {
    using acc_t = mf_f4;
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane / 16) + r; }
};

// Workgroups are handed to the 8 XCDs round-robin by id; this bijection
// gives each XCD a contiguous range of tasks, so neighbouring tasks (which
// touch neighbouring columns and rows) share that XCD's L2.
__device__ __forceinline__ int xcd_task(int bid, int ntasks) {
    constexpr int NX = 8;
    const int q = ntasks / NX, r = ntasks % NX;
    const int x = bid % NX, k = bid / NX;
    return x * q + min(x, r) + k;
}

// Cross-workgroup end of a split quadrature sum.  Every workgroup of a
// column block has stored its partial sums; one lane publishes them with a
// device-scope release (the workgroup barrier orders the other lanes' stores
// before it) and counts the arrival.  Returns true in the last workgroup to
// arrive, which then reads the others' sums (after an acquire).
__device__ __forceinline__ bool arrive_last(unsigned* counter, int n_ig, int* s_last) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(counter, 1u);
        *s_last = prev == (unsigned)(n_ig - 1);
        if (*s_last) __threadfence();
    }
    __syncthreads();
    return *s_last != 0;
}

// Load the lane's V-element share of an axis-0 column of one shifted field.
// 3D fields are stored [x0][c] (stride C between column elements); 2D fields
// are stored transposed, [c][x0], so a column is contiguous.  MIRROR (the
// real form, whose slab pass fills only the rows j0 = 0..N/2): a row j0 above
// N/2 is the conjugate of row N - j0, since the data are real.
template <class T, int N, int C, bool TRANS, bool MIRROR = false>
__device__ __forceinline__ void load_col(cx<T>* v, const cx<T>* base, int t, int c, bool active) {
    constexpr int TPT = FftShape<N>::TPT, V = FftShape<N>::V;
#pragma unroll
    for (int m = 0; m < V; ++m) {
        const int e = t + TPT * m;
        const int row = MIRROR && e > N / 2 ? N - e : e;
        const long long idx = TRANS ? (long long)c * N + row : (long long)row * C + c;
        v[m] = active ? base[idx] : cx<T>{(T)0, (T)0};
        if (MIRROR && e > N / 2) v[m].y = -v[m].y;
    }
}

// The lane's share of the axis-0 column of shift ls: the column of its slab
// field hs times the shift's own axis-0 phase factors (row ph0 of the phase
// table), which the slab pass leaves out so that shifts agreeing on the other
// axes share one slab field.
template <class T, int N, int C, bool TRANS, bool MIRROR = false>
__device__ __forceinline__ void load_shift(cx<T>* v, const cx<T>* G, int hs, const cx<T>* ph0, int t, int c,
                                           bool active) {
    constexpr int TPT = FftShape<N>::TPT, V = FftShape<N>::V;
    load_col<T, N, C, TRANS, MIRROR>(v, G + (long long)hs * N * C, t, c, active);
#pragma unroll
    for (int m = 0; m < V; ++m)
        if (active) v[m] = v[m] * ph0[t + TPT * m];
}

// ---------------------------------------------------------------------------
// Column forward transform (axis 0) of a double grid into spec0.
// ---------------------------------------------------------------------------
template <class T, int D, int N, int GB>
__global__ __launch_bounds__(GB* FftShape<N>::TPT) void k_colfwd(ColFwdArgs A) {
    using S = FftShape<N>;
    constexpr int TPT = S::TPT, V = S::V, PITCH = N + 1;
    constexpr int C = (int)ipow_c(N, D - 1);
    __shared__ cx<T> lds[GB * PITCH];
    __shared__ cx<T> tw[N];
    const TaskB task = A.tasks[xcd_task(blockIdx.x, gridDim.x)];
    const InstDev& I = A.inst[task.inst];
    const int l = threadIdx.x, g = l % GB, t = l / GB;
    const int c = task.cb * GB + g;
    const bool active = c < C;
    const cx<T>* twg = reinterpret_cast<const cx<T>*>(A.tw) + I.off_tw;
    for (int i = l; i < N; i += GB * TPT) tw[i] = twg[i];
    const double2* f = reinterpret_cast<const double2*>(A.f) + I.off_state;
    cx<T> v[V];
#pragma unroll
    for (int m = 0; m < V; ++m) {
        v[m] = active ? to_t<T>(f[(long long)(t + TPT * m) * C + c]) : cx<T>{(T)0, (T)0};
        if (I.nyq_zero) v[m].y = (T)0;        // the real form evolves Re f
    }
    fft_dist<T, N, -1>(v, lds + g * PITCH, 1, t, tw, active);
    if constexpr (S::NST == 1) __syncthreads();
    cx<T>* sp = reinterpret_cast<cx<T>*>(A.spec0) + I.off_spec0;
    const T sc = (T)I.fwd_scale;
    if (active) {
        if (D == 2 && A.spec_trans) {
#pragma unroll
            for (int m = 0; m < V; ++m) sp[(long long)c * N + t + TPT * m] = sc * v[m];
        } else {
#pragma unroll
            for (int m = 0; m < V; ++m) sp[(long long)(t + TPT * m) * C + c] = sc * v[m];
        }
    }
}

// ---------------------------------------------------------------------------
// Slab pass, 2D: a workgroup owns JB consecutive rows j0 of the axis-0
// spectrum and SB shifted fields at a time.  Each group of TPT lanes
// transforms one (row, field) pair along axis 1.  The shifted fields are
// stored transposed, G[s][x1][j0] (axis-0 index fastest), so that the
// column pass reads every column contiguously: the groups of one wavefront
// hold consecutive rows of one field, so each store instruction writes whole
// runs of JB consecutive j0 per x1.
// ---------------------------------------------------------------------------
template <class T, int N, int JB, int SB>
__global__ __launch_bounds__(JB* SB* FftShape<N>::TPT) void k_passA2d(PassAArgs A) {
    using S = FftShape<N>;
    constexpr int TPT = S::TPT, V = S::V, PITCH = scratch_slots<N>(), NT = JB * SB * TPT;
    constexpr bool WV = 64 % TPT == 0;      // a group's TPT lanes are contiguous
    __shared__ cx<T> eng[JB * SB * PITCH];
    __shared__ cx<T> fh[JB * N];
    __shared__ cx<T> tw[N];
    const TaskA task = A.tasks[xcd_task(blockIdx.x, gridDim.x)];
    const InstDev& I = A.inst[task.inst];
    const int l = threadIdx.x, gi = l / TPT, t = l % TPT;
    const int r = gi % JB, q = gi / JB;      // row within the block, field slot
    const cx<T>* twg = reinterpret_cast<const cx<T>*>(A.tw) + I.off_tw;
    for (int i = l; i < N; i += NT) tw[i] = twg[i];
    cx<T>* my = eng + gi * PITCH;
    const int j0 = task.j0 + r;
    const cx<T>* ph = reinterpret_cast<const cx<T>*>(A.ph) + I.off_ph;
    const int* hrep = A.hrep + I.off_hrep;
    // the first round's phase factors (axis 1 of the slab field's shift) are
    // fetched before the forward transform so that their latency overlaps it
    cx<T> pre[V];
    {
        const int s = task.s_begin + q;
        const cx<T>* phs = ph + (long long)hrep[s < task.s_end ? s : task.s_begin] * 2 * N;
#pragma unroll
        for (int m = 0; m < V; ++m) pre[m] = phs[N + t + TPT * m];
    }
    __syncthreads();    // twiddles in LDS
    // f_hat rows: forward transform along axis 1 of the axis-0 spectrum
    {
        const bool act = q == 0;
        const cx<T>* sp = reinterpret_cast<const cx<T>*>(A.spec0) + I.off_spec0 + (long long)j0 * N;
        cx<T> v[V];
#pragma unroll
        for (int m = 0; m < V; ++m) v[m] = act ? sp[t + TPT * m] : cx<T>{(T)0, (T)0};
        fft_dist<T, N, -1, WV, pad_scratch<N>()>(v, my, 1, t, tw, act);
        if (act) {
#pragma unroll
            for (int m = 0; m < V; ++m) fh[r * N + t + TPT * m] = v[m];
        }
    }
    __syncthreads();    // f_hat rows in LDS; from here each group uses only its own slots
    cx<T> fr[V];
#pragma unroll
    for (int m = 0; m < V; ++m) fr[m] = fh[r * N + t + TPT * m];
    cx<T>* G = reinterpret_cast<cx<T>*>(A.G) + I.off_G;
    const int nrounds = (task.s_end - task.s_begin + SB - 1) / SB;
#pragma unroll 1
    for (int round = 0; round < nrounds; ++round) {
        const int s = task.s_begin + round * SB + q;
        const bool active = s < task.s_end;
        if (round > 0) {
            const cx<T>* phs = ph + (long long)hrep[active ? s : task.s_begin] * 2 * N;
#pragma unroll
            for (int m = 0; m < V; ++m) pre[m] = phs[N + t + TPT * m];
        }
        cx<T> v[V];
#pragma unroll
        for (int m = 0; m < V; ++m) v[m] = fr[m] * pre[m];
        fft_dist<T, N, 1, WV, pad_scratch<N>()>(v, my, 1, t, tw, active);
        if (active) {
            cx<T>* Gs = G + (long long)s * N * N + j0;
#pragma unroll
            for (int m = 0; m < V; ++m) Gs[(long long)(t + TPT * m) * N] = v[m];
        }
    }
}

// ---------------------------------------------------------------------------
// Slab pass, 3D: slab j0 is an N x N plane over axes (1, 2), transformed in
// LDS and then held in registers (each lane keeps the elements its row
// transforms read); SC shifted fields are transformed at a time, each in its
// own LDS plane, the first of which is the slab's.
// ---------------------------------------------------------------------------
template <class T, int N, int GA, int SC>
__global__ __launch_bounds__(GA* FftShape<N>::TPT* SC) void k_passA3d(PassAArgs A) {
    using S = FftShape<N>;
    // rows hold at least a transform's scratch: the row transforms work in place
    constexpr int TPT = S::TPT, V = S::V, PITCH = plane_pitch<N>(sizeof(T) == 8 ? 0 : 1), NT = GA * TPT * SC,
                  SUB = GA * TPT;
    static_assert(N % GA == 0, "groups must tile the slab");
    static_assert(PITCH >= slab_row_slots<N>(), "a plane row holds a row transform's scratch");
    constexpr int SPAD = slab_row_pad<N>();
    constexpr int ROUNDS = N / GA;
    __shared__ cx<T> W[SC][N * PITCH];
    __shared__ cx<T> tw[N];
    cx<T>* const hat = W[0];
    const TaskA task = A.tasks[xcd_task(blockIdx.x, gridDim.x)];
    const InstDev& I = A.inst[task.inst];
    const int l = threadIdx.x;
    const cx<T>* twg = reinterpret_cast<const cx<T>*>(A.tw) + I.off_tw;
    for (int i = l; i < N; i += NT) tw[i] = twg[i];
    const int j0 = task.j0;
    const cx<T>* sp = reinterpret_cast<const cx<T>*>(A.spec0) + I.off_spec0 + (long long)j0 * N * N;
    for (int i = l; i < N * N; i += NT) hat[(i / N) * PITCH + (i % N)] = sp[i];
    const int sub = l / SUB, l2 = l % SUB;
    // row-pass lanes: t fastest; column-pass lanes: group fastest
    const int gr = l2 / TPT, tr = l2 % TPT;
    const int gc = l2 % GA, tc = l2 / GA;
    // Row transforms (axis 2) work in place in their own LDS row, with the
    // row's TPT lanes inside one wavefront: they order their LDS phases with
    // wavefront fences, and workgroup barriers are needed only where the
    // rows meet the column transforms (axis 1), whose lanes span wavefronts
    // (a column's lanes are GA apart, so the stores stay coalesced along x2).
    constexpr bool RW = 64 % TPT == 0;
    // forward transform of the slab over axis 2 then axis 1 (sub-block 0
    // works, the others only join the barriers)
    __syncthreads();    // slab and twiddles in LDS
#pragma unroll 1
    for (int round = 0; round < ROUNDS; ++round) {
        const int row = round * GA + gr;
        const bool act = sub == 0;
        cx<T> v[V];
        if (!RW) __syncthreads();
#pragma unroll
        for (int m = 0; m < V; ++m) v[m] = act ? hat[row * PITCH + tr + TPT * m] : cx<T>{(T)0, (T)0};
        fft_dist<T, N, -1, RW, SPAD>(v, hat + row * PITCH, 1, tr, tw, act);
        phase_sync<RW>();
        if (act) {
#pragma unroll
            for (int m = 0; m < V; ++m) hat[row * PITCH + tr + TPT * m] = v[m];
        }
    }
#pragma unroll 1
    for (int round = 0; round < ROUNDS; ++round) {
        const int col = round * GA + gc;
        const bool act = sub == 0;
        cx<T> v[V];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < V; ++m) v[m] = act ? hat[(tc + TPT * m) * PITCH + col] : cx<T>{(T)0, (T)0};
        fft_dist<T, N, -1>(v, hat + col, PITCH, tc, tw, act);
        __syncthreads();
        if (act) {
#pragma unroll
            for (int m = 0; m < V; ++m) hat[(tc + TPT * m) * PITCH + col] = v[m];
        }
    }
    // the transformed slab, in the places the field rows below read it
    // (every sub-block holds it; the barrier at the top of the field loop
    // orders these reads before plane 0 is overwritten)
    __syncthreads();    // the forward columns are written
    cx<T> hr[ROUNDS][V];
#pragma unroll
    for (int round = 0; round < ROUNDS; ++round)
#pragma unroll
        for (int m = 0; m < V; ++m) hr[round][m] = hat[(round * GA + gr) * PITCH + tr + TPT * m];
    const cx<T>* ph = reinterpret_cast<const cx<T>*>(A.ph) + I.off_ph;
    cx<T>* G = reinterpret_cast<cx<T>*>(A.G) + I.off_G;
    cx<T>* Wm = W[sub];
    const int nsr = (task.s_end - task.s_begin + SC - 1) / SC;
#pragma unroll 1
    for (int sr = 0; sr < nsr; ++sr) {
        const int s = task.s_begin + sr * SC + sub;
        const bool act = s < task.s_end;
        const cx<T>* phs = ph + (long long)A.hrep[I.off_hrep + (act ? s : task.s_begin)] * 3 * N;
        __syncthreads();    // the plane's previous columns (or the slab) have been read
#pragma unroll
        for (int round = 0; round < ROUNDS; ++round) {
            const int j1 = round * GA + gr;
            const cx<T> p01 = phs[N + j1];
            cx<T> v[V];
            if (!RW) __syncthreads();
#pragma unroll
            for (int m = 0; m < V; ++m) v[m] = hr[round][m] * (phs[2 * N + tr + TPT * m] * p01);
            fft_dist<T, N, 1, RW, SPAD>(v, Wm + j1 * PITCH, 1, tr, tw, act);
            phase_sync<RW>();
            if (act) {
#pragma unroll
                for (int m = 0; m < V; ++m) Wm[j1 * PITCH + tr + TPT * m] = v[m];
            }
        }
        cx<T>* out = G + (long long)(act ? s : 0) * N * N * N + (long long)j0 * N * N;
#pragma unroll 1
        for (int round = 0; round < ROUNDS; ++round) {
            const int x2 = round * GA + gc;
            cx<T> v[V];
            __syncthreads();
#pragma unroll
            for (int m = 0; m < V; ++m) v[m] = act ? Wm[(tc + TPT * m) * PITCH + x2] : cx<T>{(T)0, (T)0};
            fft_dist<T, N, 1>(v, Wm + x2, PITCH, tc, tw, act);
            if (act) {
#pragma unroll
                for (int m = 0; m < V; ++m) out[(long long)(tc + TPT * m) * N + x2] = v[m];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Slab pass, 3D, register form (small N): one lane holds a whole row of the
// slab and transforms it with an unrolled register DFT; rows are turned into
// columns through a per-field LDS plane, and a lane then transforms one
// column and stores it (consecutive lanes write consecutive addresses).  A
// wavefront carries 64 / N fields at a time and synchronises only with
// itself.  The slab's forward transform is done the same way by wavefront 0.
// ---------------------------------------------------------------------------
template <class T, int N, int NW>
__global__ __launch_bounds__(64 * NW) void k_passA3d_reg(PassAArgs A) {
    constexpr int PITCH = N + 1, NT = 64 * NW;
    constexpr int FPW = 64 / N;              // fields per wavefront
    static_assert(64 % N == 0, "a field's lanes must fit one wavefront");
    __shared__ cx<T> hat[N * PITCH];
    __shared__ cx<T> W[NW * FPW][N * PITCH];
    const TaskA task = A.tasks[xcd_task(blockIdx.x, gridDim.x)];
    const InstDev& I = A.inst[task.inst];
    const int l = threadIdx.x, wv = l / 64, ln = l % 64;
    const int fw = ln / N, lane = ln % N;    // field slot within the wavefront, row/column index
    const int j0 = task.j0;
    const cx<T>* sp = reinterpret_cast<const cx<T>*>(A.spec0) + I.off_spec0 + (long long)j0 * N * N;
    // forward transform of the slab: rows (lane = row), then columns
    if (wv == 0 && fw == 0) {
        cx<T> v[N];
#pragma unroll
        for (int x = 0; x < N; ++x) v[x] = sp[(long long)lane * N + x];
        dft<N, -1>(v);
#pragma unroll
        for (int x = 0; x < N; ++x) hat[lane * PITCH + x] = v[x];
    }
    __syncthreads();
    if (wv == 0 && fw == 0) {
        cx<T> v[N];
#pragma unroll
        for (int x = 0; x < N; ++x) v[x] = hat[x * PITCH + lane];
        dft<N, -1>(v);
        phase_sync<true>();   // every lane has read its column before any writes back
#pragma unroll
        for (int x = 0; x < N; ++x) hat[x * PITCH + lane] = v[x];
    }
    __syncthreads();
    const cx<T>* ph = reinterpret_cast<const cx<T>*>(A.ph) + I.off_ph;
    cx<T>* G = reinterpret_cast<cx<T>*>(A.G) + I.off_G;
    cx<T>* Wm = W[wv * FPW + fw];
    constexpr int PER = NW * FPW;            // fields in flight per workgroup
    const int slot = wv * FPW + fw;
#pragma unroll 1
    for (int s0 = task.s_begin; s0 < task.s_end; s0 += PER) {
        const int s = s0 + slot;
        const bool act = s < task.s_end;
        const cx<T>* phs = ph + (long long)A.hrep[I.off_hrep + (act ? s : task.s_begin)] * 3 * N;
        // row j1 = lane: phase multiply, inverse transform along axis 2
        const cx<T> p01 = phs[N + lane];
        cx<T> v[N];
#pragma unroll
        for (int x = 0; x < N; ++x) v[x] = hat[lane * PITCH + x] * (phs[2 * N + x] * p01);
        dft<N, 1>(v);
        phase_sync<true>();   // the plane's previous columns have been read
#pragma unroll
        for (int x = 0; x < N; ++x) Wm[lane * PITCH + x] = v[x];
        phase_sync<true>();
        // column x2 = lane: inverse transform along axis 1, then store
#pragma unroll
        for (int x = 0; x < N; ++x) v[x] = Wm[x * PITCH + lane];
        dft<N, 1>(v);
        if (act) {
            cx<T>* out = G + (long long)s * N * N * N + (long long)j0 * N * N;
#pragma unroll
            for (int x = 0; x < N; ++x) out[(long long)x * N + lane] = v[x];
        }
    }
}

// ---------------------------------------------------------------------------
// Column pass: shifted fields on the grid, products, weighted sums, epilogue.
// A workgroup owns GB columns of axis 0 and runs IGS quadrature items at a
// time ("item slots", one per group of GB*TPT lanes); the slots' sums are
// combined in LDS in a fixed order, then (when the items of a column block
// are split over several workgroups) across workgroups through a partial
// buffer, the last arriving workgroup finishing the block.
// ---------------------------------------------------------------------------
template <class T, int D, int N, int GB, int IGS, int MODE>
__global__ __launch_bounds__(GB* FftShape<N>::TPT* IGS) void k_passB(PassBArgs A) {
    using S = FftShape<N>;
    constexpr int TPT = S::TPT, V = S::V, PITCH = scratch_slots<N>();
    constexpr int C = (int)ipow_c(N, D - 1);
    constexpr long long NP = ipow_c(N, D);
    constexpr int SLOT = GB * TPT;
    constexpr bool WV = SLOT <= 64 && 64 % SLOT == 0;   // a slot's transforms live in one wavefront
    constexpr bool TRANS = D == 2;                      // 2D fields are stored column-contiguous
    constexpr size_t FFT_BYTES = sizeof(cx<T>) * IGS * GB * PITCH;
    constexpr size_t RED_BYTES = sizeof(double2) * (IGS > 1 ? IGS / 2 : 1) * GB * N;
    constexpr size_t SMEM = FFT_BYTES > RED_BYTES ? FFT_BYTES : RED_BYTES;
    __shared__ __align__(16) unsigned char smem[SMEM];
    __shared__ cx<T> tw[N];
    __shared__ int hidl[HID_CAP];
    __shared__ int s_last;
    const TaskB task = A.tasks[xcd_task(blockIdx.x, gridDim.x)];
    const InstDev& I = A.inst[task.inst];
    const int l = threadIdx.x;
    const int slot = l / SLOT, r = l % SLOT;
    const int g = r % GB, t = r / GB;
    const int c = task.cb * GB + g;
    const bool col_ok = c < C;
    const cx<T>* twg = reinterpret_cast<const cx<T>*>(A.tw) + I.off_tw;
    for (int i = l; i < N; i += SLOT * IGS) tw[i] = twg[i];
    const int it0 = task.ig * I.items_per_ig;
    const int it1 = min(I.n_items, it0 + I.items_per_ig);
    {
        const int* hid = A.hid + I.off_hid + (long long)it0 * I.S_item;
        for (int i = l; i < (it1 - it0) * I.S_item; i += SLOT * IGS) hidl[i] = hid[i];
    }
    cx<T>* my = reinterpret_cast<cx<T>*>(smem) + (slot * GB + g) * PITCH;
    __syncthreads();    // twiddles and slab-field indices in LDS

    cx<T> F0[V];
    {
        const double2* fp = reinterpret_cast<const double2*>(A.F0) + I.off_state;
#pragma unroll
        for (int m = 0; m < V; ++m)
            F0[m] = col_ok ? to_t<T>(fp[(long long)(t + TPT * m) * C + c]) : cx<T>{(T)0, (T)0};
    }
    cx<T> acc[V], cmp[V];
#pragma unroll
    for (int m = 0; m < V; ++m) acc[m] = cmp[m] = cx<T>{(T)0, (T)0};

    const cx<T>* G = reinterpret_cast<const cx<T>*>(A.G) + I.off_G;
    const cx<T>* ph = reinterpret_cast<const cx<T>*>(A.ph) + I.off_ph;
    const T* uw = reinterpret_cast<const T*>(A.uw) + I.off_unit;
    const UnitPat* up = A.upat + A.upat_off[task.inst];
    const int rounds = (it1 - it0 + IGS - 1) / IGS;
    const int SI = I.S_item;
    const long long prow = (long long)D * N;     // phase-table row of one shift
    const int nu = I.U_item;
    // units are processed in batches of UB whose column loads are issued
    // together, so the memory latency is paid once per batch
    constexpr int UB = sizeof(T) == 8 ? (SLOT * IGS <= 128 ? 2 : 1) : (SLOT * IGS > 256 ? 2 : 4);
#pragma unroll 1
    for (int k = 0; k < rounds; ++k) {
        const int it = it0 + k * IGS + slot;
        const bool active = col_ok && it < it1;
        const int il = (it < it1 ? it : it0) - it0;       // item within the workgroup's range
        const int* hi = hidl + il * SI;
        const cx<T>* phi = ph + (long long)(it0 + il) * SI * prow;
        cx<T> a[V];
        cx<T> bq[UB][V], cq[UB][V];
        load_shift<T, N, C, TRANS>(a, G, hi[0], phi, t, c, active);
#pragma unroll
        for (int j = 0; j < UB; ++j) {
            if (j < nu) {
                const UnitPat p = up[j];
                load_shift<T, N, C, TRANS>(bq[j], G, hi[p.b], phi + p.b * prow, t, c, active);
                load_shift<T, N, C, TRANS>(cq[j], G, hi[p.c], phi + p.c * prow, t, c, active);
            }
        }
        fft_dist<T, N, 1, WV, pad_scratch<N>()>(a, my, 1, t, tw, active);
#pragma unroll 1
        for (int u0 = 0; u0 < nu; u0 += UB) {
            if (u0 > 0) {
#pragma unroll
                for (int j = 0; j < UB; ++j) {
                    if (u0 + j < nu) {
                        const UnitPat p = up[u0 + j];
                        load_shift<T, N, C, TRANS>(bq[j], G, hi[p.b], phi + p.b * prow, t, c, active);
                        load_shift<T, N, C, TRANS>(cq[j], G, hi[p.c], phi + p.c * prow, t, c, active);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < UB; ++j) {
                const int u = u0 + j;
                if (u < nu) {
                    const T w = active ? uw[(long long)it * nu + u] : (T)0;
                    fft_dist<T, N, 1, WV, pad_scratch<N>()>(bq[j], my, 1, t, tw, active);
                    fft_dist<T, N, 1, WV, pad_scratch<N>()>(cq[j], my, 1, t, tw, active);
#pragma unroll
                    for (int m = 0; m < V; ++m) {
                        // b c (a + F0) - F0 a (b + c) = abc - F0 ac + b F0 c - b a F0
                        const cx<T> b = bq[j][m], cc = cq[j][m];
                        const cx<T> bc = b * cc;
                        const cx<T> P = bc * (a[m] + F0[m]) - (F0[m] * a[m]) * (b + cc);
                        acc_add(acc[m].x, cmp[m].x, w * P.x);
                        acc_add(acc[m].y, cmp[m].y, w * P.y);
                    }
                }
            }
        }
    }

    // the RK epilogue's inputs are fetched now, so their latency overlaps
    // the slot reduction
    const bool lead = slot == 0 && col_ok;   // lanes that own the block's results
    double2 yb[V], kb[V];
    if (MODE == MODE_RK && lead) {
        const double2* y = reinterpret_cast<const double2*>(A.y) + I.off_state;
        const double2* ks = reinterpret_cast<const double2*>(A.ksum) + I.off_state;
#pragma unroll
        for (int m = 0; m < V; ++m) {
            const long long idx = (long long)(t + TPT * m) * C + c;
            yb[m] = y[idx];
            kb[m] = A.stage == 0 ? make_double2(0.0, 0.0) : ks[idx];
        }
    }

    // combine the item slots in LDS by a fixed pairwise tree: at each level
    // slot k adds slot k + h
    double2 sum[V];
#pragma unroll
    for (int m = 0; m < V; ++m) sum[m] = make_double2((double)acc[m].x + (double)cmp[m].x,
                                                      (double)acc[m].y + (double)cmp[m].y);
    if constexpr (IGS > 1) {
        static_assert((IGS & (IGS - 1)) == 0, "item slots must be a power of two");
        double2* red = reinterpret_cast<double2*>(smem);
#pragma unroll
        for (int h = IGS / 2; h >= 1; h /= 2) {
            __syncthreads();    // the transforms' (or the previous level's) LDS use is over
            if (slot >= h && slot < 2 * h) {
#pragma unroll
                for (int m = 0; m < V; ++m) red[((slot - h) * GB + g) * N + t + TPT * m] = sum[m];
            }
            __syncthreads();
            if (slot < h) {
#pragma unroll
                for (int m = 0; m < V; ++m) {
                    const double2 v = red[(slot * GB + g) * N + t + TPT * m];
                    sum[m].x += v.x;
                    sum[m].y += v.y;
                }
            }
        }
    }
    if (I.n_ig > 1) {
        double2* part = reinterpret_cast<double2*>(A.part) + I.off_part;
        if (lead) {
#pragma unroll
            for (int m = 0; m < V; ++m) part[task.ig * NP + (long long)(t + TPT * m) * C + c] = sum[m];
        }
        if (!arrive_last(&A.counters[I.counter_off + task.cb], I.n_ig, &s_last)) return;
#pragma unroll
        for (int m = 0; m < V; ++m) sum[m] = make_double2(0.0, 0.0);
        if (lead) {
            // two item groups' partial sums in flight at a time, added in order
            for (int ig = 0; ig < I.n_ig; ig += 2) {
                const bool two = ig + 1 < I.n_ig;
                double2 r0[V], r1[V];
#pragma unroll
                for (int m = 0; m < V; ++m) {
                    const double* src = reinterpret_cast<const double*>(part + ig * NP + (long long)(t + TPT * m) * C + c);
                    r0[m].x = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    r0[m].y = __hip_atomic_load(src + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    r1[m] = make_double2(0.0, 0.0);
                    if (two) {
                        r1[m].x = __hip_atomic_load(src + 2 * NP, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        r1[m].y = __hip_atomic_load(src + 2 * NP + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
#pragma unroll
                for (int m = 0; m < V; ++m) {
                    sum[m].x += r0[m].x;
                    sum[m].y += r0[m].y;
                    if (two) {
                        sum[m].x += r1[m].x;
                        sum[m].y += r1[m].y;
                    }
                }
            }
        }
        if (l == 0) A.counters[I.counter_off + task.cb] = 0u;
    }

    const double qs = I.q_scale;
    if constexpr (MODE == MODE_EVAL) {
        if (lead) {
            double2* out = reinterpret_cast<double2*>(A.out) + I.off_state;
#pragma unroll
            for (int m = 0; m < V; ++m)
                out[(long long)(t + TPT * m) * C + c] = make_double2(qs * sum[m].x, qs * sum[m].y);
        }
        return;
    } else {
        // classical RK4 stage update, then the axis-0 forward transform of the
        // next stage state for the following slab pass
        double2* y = reinterpret_cast<double2*>(A.y) + I.off_state;
        double2* ys = reinterpret_cast<double2*>(A.ystage) + I.off_state;
        double2* ks = reinterpret_cast<double2*>(A.ksum) + I.off_state;
        const double dt = A.dt;
        cx<T> nxt[V];
#pragma unroll
        for (int m = 0; m < V; ++m) {
            nxt[m] = cx<T>{(T)0, (T)0};
            if (!lead) continue;
            const long long idx = (long long)(t + TPT * m) * C + c;
            const double kx = qs * sum[m].x, ky = qs * sum[m].y;
            const double2 y0 = yb[m], k0 = kb[m];
            double2 ns;
            if (A.stage == 0) {
                ks[idx] = make_double2(kx, ky);
                ns = make_double2(y0.x + 0.5 * dt * kx, y0.y + 0.5 * dt * ky);
                ys[idx] = ns;
            } else if (A.stage == 1 || A.stage == 2) {
                ks[idx] = make_double2(k0.x + 2.0 * kx, k0.y + 2.0 * ky);
                const double cst = A.stage == 1 ? 0.5 * dt : dt;
                ns = make_double2(y0.x + cst * kx, y0.y + cst * ky);
                ys[idx] = ns;
            } else {
                ns = make_double2(y0.x + dt / 6.0 * (k0.x + kx), y0.y + dt / 6.0 * (k0.y + ky));
                y[idx] = ns;
            }
            nxt[m] = to_t<T>(ns);
        }
        __syncthreads();        // the reduction area is about to be reused
        fft_dist<T, N, -1, WV, pad_scratch<N>()>(nxt, my, 1, t, tw, lead);
        if (lead) {
            cx<T>* sp = reinterpret_cast<cx<T>*>(A.spec0) + I.off_spec0;
            const T sc = (T)I.fwd_scale;
#pragma unroll
            for (int m = 0; m < V; ++m) sp[(long long)(t + TPT * m) * C + c] = sc * nxt[m];
        }
    }
}

// ---------------------------------------------------------------------------
// Column pass, field-parallel form.  One workgroup per block of GB
// neighbouring columns of axis 0 (one column in 2D, whose columns are
// contiguous; 4 in 3D, so that a field's loads are 64-byte runs) and item
// group.  Shifts that coincide as vectors across the quadrature items are one
// field: every distinct field of the workgroup's items gets its own block of
// GB x TPT lanes (column fastest), so all of them are transformed at once and
// each only once.  The transformed columns stay in LDS; the products and the
// weighted sum are then taken point by point, KP = blockDim / (GB N) lanes
// per point, each over its own items in order, and the KP sums are added in
// a fixed order.  When the fields of all the items do not fit, items are
// taken in rounds (built on the host) whose fields do.
// Dynamic LDS: the field columns [fields][slots][GB] during the rounds (the
// GB columns of a field interleaved); then the per-lane sums [KP][GB N]
// (double2), the next stage state [N][GB] and the scratch of its transforms
// [slots][GB].
// ---------------------------------------------------------------------------
// FUSED (2D): before the rounds, the workgroup builds the slab-field columns
// of its column c itself: H_h(j0, c) = sum over x1 of spec0(j0, x1) K_h(c - x1),
// K_h the axis-1 interpolation kernel of slab field h (the inverse DFT of its
// axis-1 phase row).  The sum over x1 is split in fp_nwp chunks, each a lane
// per j0 holding every slab field's partial sum; spec0 is stored [x1][j0],
// so a chunk's loads are contiguous.
// REAL (the Nyquist-zero real form): every field is real, so each lane
// block transforms two round-local fields 2bi and 2bi+1 as one complex
// column (the first in the real part, the second in the imaginary part),
// the products are real, and the unshifted factor F0 is the round's local
// field 0, the zero shift, which carries the state with its Nyquist modes
// dropped.
template <class T, int D, int N, int MODE, int FUS, bool REAL, bool ONE>
__global__ __launch_bounds__(fp_max_threads(sizeof(T) == 8 ? 0 : 1, N, FUS != 0, REAL)) void k_passB_fp(PassBArgs A) {
    // FUS: 0 the field-parallel form, 1 fused with the vector interpolation,
    // 2 fused with the matrix-core interpolation (separate instances: each
    // carries only its own interpolation code, and a smaller kernel loses
    // less time to instruction fetch at the start of every launch).  ONE: a
    // single-instance plan with one item group, whose tasks differ only in
    // their column block, the task's place in the list: the task comes from
    // the kernel arguments and the descriptor is read at once, so the tables
    // and operands are requested one or two dependent loads earlier (the
    // fused forms only)
    constexpr bool FUSED = FUS != 0;
    using S = FftShape<N>;
    constexpr int TPT = S::TPT, V = S::V, PITCH = col_slots<D, N>(), CPAD = col_pad<D, N>();
    constexpr int GB = fp_block(D), BLK = GB * TPT, P = GB * N;
    constexpr int C = (int)ipow_c(N, D - 1);
    constexpr long long NP = ipow_c(N, D);
    constexpr bool WV = BLK <= 64 && 64 % BLK == 0;     // a field block's transforms share a wavefront
    constexpr bool TRANS = D == 2;                      // 2D fields are stored column-contiguous
    static_assert(!FUSED || D == 2, "the fused form is 2D");
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ cx<T> tw[N];
    __shared__ T wts[FP_MAX_GROUPS];
    // per item, the LDS offsets (from a point's own slot) of its factor a and
    // of b and c of each unit in unit order, written by the host: a unit
    // costs one read of its two offsets and two value reads, with no index
    // arithmetic beyond two shifted adds
    __shared__ int uofs_l[HID_CAP];
    __shared__ FieldRef fld_l[HID_CAP];          // the rounds' fields: (defining shift, slab field)
    __shared__ int s_last;
    cx<T>* fb = reinterpret_cast<cx<T>*>(dyn);
    const TaskB task = ONE ? TaskB{0, xcd_task(blockIdx.x, gridDim.x), 0, A.task1.r0, A.task1.r1, A.task1.f0,
                                   A.task1.nfl, A.task1.sub}
                           : A.tasks[xcd_task(blockIdx.x, gridDim.x)];
    const InstDev& I = A.inst[ONE ? 0 : task.inst];
    const int l = threadIdx.x, NT = blockDim.x;
    const int bi = l / BLK, rl = l % BLK, g = rl % GB, t = rl / GB;   // field block, its column, transform lane
    const int KP = NT / P;
    const int pp = l % P, kq = l / P;        // product phase: point pp of the block, lane kq of its KP
    const int pg = pp % GB, x = pp / GB;     // ... its column and its index along axis 0
    const bool prod = kq < KP, lead = l < P;
    const int c = task.cb * GB + g, cp = task.cb * GB + pg;
    const bool col_ok = c < C, colp_ok = cp < C;
    const int Sf = I.S_item, U = I.U_item;
    const cx<T>* twg = reinterpret_cast<const cx<T>*>(A.tw) + I.off_tw;
    for (int i = l; i < N; i += NT) tw[i] = twg[i];
    const int it0 = task.ig * I.items_per_ig;
    const int it1 = min(I.n_items, it0 + I.items_per_ig);
    {
        const int* uo = A.uofs + I.off_hid + (long long)it0 * Sf;
        for (int i = l; i < (it1 - it0) * Sf; i += NT) uofs_l[i] = uo[i];
        const FieldRef* fl = A.flds + I.off_hid + task.f0;
        for (int i = l; i < task.nfl; i += NT) fld_l[i] = fl[i];
    }
    // FUSED: the slab-field columns [slab field][HP] of column c, the
    // interpolation partial sums [part][slab field][PP] and the staged phase
    // rows [block][NPF][HP], rows padded so that the field blocks of a
    // wavefront, and the slab fields of a matrix-core tile, fall on
    // different LDS banks
    constexpr int HP = fused_hpitch(N), PP = fused_ppitch(sizeof(T) == 8 ? 0 : 1, N);
    cx<T>* Hb = reinterpret_cast<cx<T>*>(dyn + A.fp_off_h);
    // FUSED: the slab fields this item group's items use, the rounds' fields
    // naming them by their place in the list (task.sub < 0: all of the
    // instance's slab fields in order, so no list needs to be read first)
    const bool ident = task.sub < 0;
    const int* subl = FUSED && !ident ? A.sub + task.sub + 1 : nullptr;
    const int nsub = FUSED ? (ident ? I.n_slab : A.sub[task.sub]) : 0;
    // FUSED: every load the interpolation needs is issued here, with the
    // tables, so that their latencies overlap before the first barrier: this
    // column's interpolation kernels, Kp[h][x] = K_h((c - x) mod N), gathered
    // into LDS after the slab-field columns (unless they are read into scalar
    // registers, KSGPR), and the lane's first batch of spectrum values into
    // registers
    constexpr int XB = 8;
    // double with N a multiple of 64: a chunk of the interpolation sum is
    // whole wavefronts, so the kernel values K_h(c - x) a wavefront needs
    // are the same for all its lanes and are read from the doubled table
    // straight into scalar registers (measured faster in double than the
    // LDS broadcast, slower in float)
    constexpr bool KSGPR = FUSED && N % 64 == 0 && sizeof(T) == 8;
    const int nwp = FUSED ? A.fp_nwp : 1;
    int hb = 0, he = nsub, lr = l;                              // the lane's slab fields [hb, he)
    bool on = FUSED && l < nwp * N;
    if constexpr (FUSED && sizeof(T) == 4) {
        // float: the lanes beyond the nwp x N of one pass take a share of
        // the slab fields each, so that every lane works (+2% per evaluation
        // at N = 64; in double the extra registers spill, so there one pass
        // of lanes does all the fields)
        const int nsh = NT / (nwp * N);                         // >= 1 (fused_chunks)
        const int fsh = (nsub + nsh - 1) / nsh;                 // slab fields per share
        const int sh = l / (nwp * N);
        lr = l % (nwp * N);
        hb = sh * fsh;
        he = min(nsub, hb + fsh);
        on = sh < nsh && hb < he;
    }
    constexpr bool mfma = FUS == 2;
    if (mfma) on = false;
    const int xs = N / nwp, w_ch = lr / N, j_ch = lr % N;       // chunk of the sum, spectrum row j0
    const cx<T>* Sx = reinterpret_cast<const cx<T>*>(A.spec0) + I.off_spec0 + j_ch;   // spec0[x1][j0]
    cx<T> sv0[XB];
    if constexpr (FUSED) {
        if (mfma) {
            // Matrix-core interpolation.  For this column, with S = spec0
            // [x1][j0] and K_h the slab field's interpolation kernel:
            //   Re H_h(j0) = sum_x Re S Re K_h(c - x) - Im S Im K_h(c - x),
            //   Im H_h(j0) = sum_x Re S Im K_h(c - x) + Im S Re K_h(c - x),
            // a real GEMM with rows j0, columns n = 2 h + (0 real, 1
            // imaginary part) and depth (x, part).  Each group of four x
            // values is two 16 x 16 x 4 steps: the real parts of S against
            // (Re K, Im K), then the imaginary parts against (-Im K, Re K).
            // A wavefront takes one (tile, depth part); its operands come
            // straight from global memory into registers (no LDS, no
            // barrier), all issued at once.  The partial tiles go to pr
            // [part][slab field][j0], summed with the other parts below.
            using M = Mfma<T>;
            constexpr int XG = N / 4;                                // groups of four x values
            const int MT = N / 16, TT = mfma_tiles(N, nsub), KS = nwp, xg = XG / KS;
            const int wv = l / 64, ln = l % 64, q = ln / 16, col = ln % 16;
            const cx<T>* K2 = reinterpret_cast<const cx<T>*>(A.kt) + I.off_kt;   // [slab field][2N]
            T* prT = reinterpret_cast<T*>(dyn);
#pragma unroll 1
            for (int u = wv; u < TT * KS; u += NT / 64) {
                const int tile = u % TT, ks = u / TT;
                const int mt = tile % MT, nt = tile / MT;
                const int j0 = 16 * mt + col;                        // this lane's A row
                const int h = 8 * nt + col / 2, part = col & 1;     // this lane's B column
                const bool hv = h < nsub;
                const cx<T>* Kr = K2 + (long long)(hv ? (ident ? h : subl[h]) : 0) * 2 * N + N + c;
                const int x0 = ks * xg * 4 + q;
                typename M::acc_t acc = {0, 0, 0, 0};
                // operands in flight (fewer in double: sixteen groups of
                // double operands would not fit a 1024-lane workgroup's
                // registers; at the headline shape a wavefront's depth part
                // is eight groups, so they all go out at once either way)
                constexpr int PFM = sizeof(T) == 8 ? 8 : 16, PF = XG < PFM ? XG : PFM;
#pragma unroll 1
                for (int g0 = 0; g0 < xg; g0 += PF) {
                    cx<T> av[PF], bv[PF];
#pragma unroll
                    for (int g = 0; g < PF; ++g) {
                        const int x = x0 + 4 * (g0 + g);
                        const bool ok = g0 + g < xg;
                        av[g] = ok ? Sx[(long long)x * N - j_ch + j0] : cx<T>{(T)0, (T)0};
                        bv[g] = ok && hv ? Kr[-x] : cx<T>{(T)0, (T)0};
                    }
#pragma unroll
                    for (int g = 0; g < PF; ++g) {
                        acc = M::step(av[g].x, part ? bv[g].y : bv[g].x, acc);
                        acc = M::step(av[g].y, part ? bv[g].x : -bv[g].y, acc);
                    }
                }
                if (hv) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        prT[2 * (((long long)ks * nsub + h) * PP + 16 * mt + M::row(ln, r)) + part] = acc[r];
                }
            }
        }
        const cx<T>* kt = reinterpret_cast<const cx<T>*>(A.kt) + I.off_kt;
        cx<T>* Kp = Hb + nsub * HP;
        if (!mfma && !KSGPR)
            for (int i = l; i < nsub * N; i += NT) {
                const int h = i / N, xx = i % N;
                Kp[i] = kt[(ident ? h : subl[h]) * 2 * N + (c - xx + N) % N];
            }
#pragma unroll
        for (int k = 0; k < XB; ++k)
            sv0[k] = on && !KSGPR ? Sx[(long long)(w_ch * xs + k) * N] : cx<T>{(T)0, (T)0};
    }
    const long long pidx = (long long)x * C + cp;  // grid index of the lane's point
    cx<T> F0 = {(T)0, (T)0};
    if (!REAL && prod && colp_ok) F0 = to_t<T>(reinterpret_cast<const double2*>(A.F0)[I.off_state + pidx]);
    double2 yb = make_double2(0.0, 0.0), kb = make_double2(0.0, 0.0);
    if (MODE == MODE_RK && lead && colp_ok) {
        yb = reinterpret_cast<const double2*>(A.y)[I.off_state + pidx];
        if (A.stage != 0) kb = reinterpret_cast<const double2*>(A.ksum)[I.off_state + pidx];
    }
    const cx<T>* G = reinterpret_cast<const cx<T>*>(A.G) + I.off_G;
    const cx<T>* ph = reinterpret_cast<const cx<T>*>(A.ph) + I.off_ph;
    const T* uw = reinterpret_cast<const T*>(A.uw) + I.off_unit;
    T ax = (T)0, ay = (T)0, ex = (T)0, ey = (T)0;   // sums and their compensations
    const RoundDesc* rds = A.rounds + I.off_rounds;
    // Fused: the axis-0 phase rows of the block's first-round field(s) are
    // copied to LDS now (when the plan has room, fp_off_ph), so that their
    // loads overlap the table loads and the interpolation instead of
    // following it.  The item group's field list starts with its first
    // round's, so the fields are read at task.f0.
    constexpr int NPF = REAL ? 2 : 1;                           // staged rows per block
    cx<T>* Pst = reinterpret_cast<cx<T>*>(dyn + A.fp_off_ph);   // [block][NPF][HP]
    if constexpr (FUSED) {
        if (A.fp_off_ph && task.r0 < task.r1) {
            const int k0 = REAL ? 2 * bi : bi;
            const int nf0 = rds[task.r0].nf;
            const FieldRef* fl = A.flds + I.off_hid + task.f0;
#pragma unroll
            for (int q = 0; q < NPF; ++q) {
                if (k0 + q < nf0) {
                    const cx<T>* p0 = ph + (long long)fl[k0 + q].x * 2 * N;
#pragma unroll
                    for (int m = 0; m < V; ++m) Pst[(bi * NPF + q) * HP + t + TPT * m] = p0[t + TPT * m];
                }
            }
        }
    }
    __syncthreads();    // twiddles, factor offsets and field tables in LDS
    if constexpr (FUSED) {
        const int ns = nsub;
        const cx<T>* Kp = Hb + ns * HP;
        cx<T>* pr = reinterpret_cast<cx<T>*>(dyn);               // [chunk][slab field][j0] partial sums
        if (on) {
            // XB spectrum values at a time (the first batch prefetched above),
            // each used for every slab field (HS per sweep, the kernel values
            // broadcast from LDS, or in scalar registers) before the next
            // batch; the partial sums of the batches carry over in LDS
            constexpr int HS = sizeof(T) == 8 ? (KSGPR ? 3 : 4) : 8;
            const cx<T>* K2 = reinterpret_cast<const cx<T>*>(A.kt) + I.off_kt;   // [slab field][2N]
            // (the first batch is peeled so that sv0 stays in registers)
            auto batch = [&](const cx<T>(&sv)[XB], int xb) {
                const int xa = w_ch * xs + xb;
                const int xau = KSGPR ? __builtin_amdgcn_readfirstlane(xa) : xa;   // uniform per wavefront
#pragma unroll 1
                for (int h0 = hb; h0 < he; h0 += HS) {
                    cx<T> acc[HS];
#pragma unroll
                    for (int h = 0; h < HS; ++h)
                        acc[h] = xb > 0 && h0 + h < he ? pr[(w_ch * ns + h0 + h) * PP + j_ch] : cx<T>{(T)0, (T)0};
#pragma unroll
                    for (int h = 0; h < HS; ++h) {
                        if (h0 + h < he) {
                            if constexpr (KSGPR) {
                                const int hk = ident ? h0 + h : subl[h0 + h];
                                const cx<T>* kr = K2 + (long long)hk * 2 * N + N + c - xau;
#pragma unroll
                                for (int k = 0; k < XB; ++k) acc[h] = acc[h] + kr[-k] * sv[k];
                            } else {
                                const cx<T>* kr = Kp + (h0 + h) * N + xa;
#pragma unroll
                                for (int k = 0; k < XB; ++k) acc[h] = acc[h] + kr[k] * sv[k];
                            }
                        }
                    }
#pragma unroll
                    for (int h = 0; h < HS; ++h)
                        if (h0 + h < he) pr[(w_ch * ns + h0 + h) * PP + j_ch] = acc[h];
                }
            };
            if constexpr (KSGPR) {
                // (not prefetched: its registers would be held across the
                // barrier, where this form has none to spare)
#pragma unroll
                for (int k = 0; k < XB; ++k) sv0[k] = Sx[(long long)(w_ch * xs + k) * N];
            }
            batch(sv0, 0);
#pragma unroll 1
            for (int xb = XB; xb < xs; xb += XB) {
                cx<T> sv[XB];
#pragma unroll
                for (int k = 0; k < XB; ++k) sv[k] = Sx[(long long)(w_ch * xs + xb + k) * N];
                batch(sv, xb);
            }
        }
        __syncthreads();
        for (int i = l; i < ns * N; i += NT) {
            const int h = i / N, j = i % N;
            cx<T> sum = pr[h * PP + j];
            for (int w = 1; w < nwp; ++w) sum = sum + pr[(w * ns + h) * PP + j];
            Hb[h * HP + j] = sum;
        }
        __syncthreads();    // slab-field columns in LDS; the partial sums are done with
    }
#pragma unroll 1
    for (int rr = task.r0; rr < task.r1; ++rr) {
        const RoundDesc R = rds[rr];
        const int ni = R.ib - R.ia;
        const int k0 = REAL ? 2 * bi : bi;     // the block's (first) round-local field
        const bool act = k0 < R.nf;
        if (l < ni * U) wts[l] = uw[(long long)R.ia * U + l];
        // column of one field: its slab field times its axis-0 phases
        auto load_field = [&](cx<T>* dst, int k, bool on) {
            const FieldRef fd = fld_l[R.foff - task.f0 + (on ? k : 0)];
            if constexpr (FUSED) {
                // the first round's phases were staged in LDS (see above)
                const bool st = A.fp_off_ph && rr == task.r0;
                const cx<T>* p0 = st ? Pst + (bi * NPF + (k - k0)) * HP : ph + (long long)fd.x * 2 * N;
#pragma unroll
                for (int m = 0; m < V; ++m)
                    dst[m] = on ? Hb[fd.y * HP + t + TPT * m] * p0[t + TPT * m] : cx<T>{(T)0, (T)0};
            } else {
                load_shift<T, N, C, TRANS, REAL>(dst, G, fd.y, ph + (long long)fd.x * D * N, t, c, on && col_ok);
            }
        };
        cx<T> v[V];
        load_field(v, k0, act);
        if constexpr (REAL) {
            // the second field rides in the imaginary part: v + i w, added
            // element by element so that its column is never held whole
            const bool act2 = act && k0 + 1 < R.nf;
            const FieldRef f2 = fld_l[R.foff - task.f0 + (act2 ? k0 + 1 : 0)];
#pragma unroll
            for (int m = 0; m < V; ++m) {
                const int e = t + TPT * m;
                cx<T> w = {(T)0, (T)0};
                if constexpr (FUSED) {
                    if (act2) {
                        const cx<T> p = A.fp_off_ph && rr == task.r0 ? Pst[(bi * NPF + 1) * HP + e]
                                                                    : ph[(long long)f2.x * 2 * N + e];
                        w = Hb[f2.y * HP + e] * p;
                    }
                } else if (act2 && col_ok) {
                    // rows above N/2 are the conjugates of rows N - j0 (see load_col)
                    const int row = e > N / 2 ? N - e : e;
                    const cx<T>* base = G + (long long)f2.y * N * C;
                    w = base[TRANS ? (long long)c * N + row : (long long)row * C + c];
                    if (e > N / 2) w.y = -w.y;
                    w = w * ph[(long long)f2.x * D * N + e];
                }
                v[m] = cx<T>{v[m].x - w.y, v[m].y + w.x};
            }
        }
        // the GB columns of a field block share one scratch, interleaved
        // element by element (column g at offset g, stride GB): the lanes of
        // a block, columns fastest, then fall on different LDS banks in
        // every phase of the transform, and the product phase's lanes, one
        // point each, read consecutive slots
        cx<T>* my = fb + bi * GB * PITCH + g;
        fft_dist<T, N, 1, WV, CPAD>(v, my, GB, t, tw, act);
        phase_sync<WV>();   // the block's last reads of its slots are done
        if (act) {
#pragma unroll
            for (int m = 0; m < V; ++m) my[(t + TPT * m) * GB] = v[m];
        }
        __syncthreads();
        // the point's own slot in block 0, from which the factor offsets
        // count (in complex slots, or in the real form in components of T;
        // typed, so that each value is one aligned LDS access)
        const cx<T>* fpt = fb + x * GB + pg;
        const T* fpr = reinterpret_cast<const T*>(fpt);
        if (REAL && prod) {
            const T F0r = fpr[0];   // round-local field 0, the zero shift
#pragma unroll 1
            for (int ii = kq; ii < ni; ii += KP) {
                const int* uo = uofs_l + (R.ia + ii - it0) * Sf;
                const T a = fpr[uo[0]];
                // sum over the item's units of w [b c (a + F0) - F0 a (b + c)]
                // = (a + F0) sum w b c - F0 a sum w (b + c)
                T s1 = (T)0, s2 = (T)0;
#pragma unroll 2
                for (int u = 0; u < U; ++u) {
                    const T b = fpr[uo[1 + 2 * u]], cc = fpr[uo[2 + 2 * u]], w = wts[ii * U + u];
                    s1 += w * (b * cc);
                    s2 += w * (b + cc);
                }
                acc_add(ax, ex, (a + F0r) * s1 - (F0r * a) * s2);
            }
        } else if (prod) {
#pragma unroll 1
            for (int ii = kq; ii < ni; ii += KP) {
                const int* uo = uofs_l + (R.ia + ii - it0) * Sf;
                const cx<T> a = fpt[uo[0]];
                // sum over the item's units of w [b c (a + F0) - F0 a (b + c)]
                // = (a + F0) sum w b c - F0 a sum w (b + c)
                cx<T> s1 = {(T)0, (T)0}, s2 = {(T)0, (T)0};
#pragma unroll 2
                for (int u = 0; u < U; ++u) {
                    const cx<T> b = fpt[uo[1 + 2 * u]], cc = fpt[uo[2 + 2 * u]];
                    const T w = wts[ii * U + u];
                    const cx<T> bc = b * cc;
                    s1 = cx<T>{s1.x + w * bc.x, s1.y + w * bc.y};
                    s2 = cx<T>{s2.x + w * (b.x + cc.x), s2.y + w * (b.y + cc.y)};
                }
                const cx<T> Pv = (a + F0) * s1 - (F0 * a) * s2;
                acc_add(ax, ex, Pv.x);
                acc_add(ay, ey, Pv.y);
            }
        }
        __syncthreads();    // the round's columns and weights are consumed
    }

    double2* red = reinterpret_cast<double2*>(dyn);
    if (prod) red[kq * P + pp] = make_double2((double)ax + (double)ex, (double)ay + (double)ey);
    __syncthreads();
    double2 sum = make_double2(0.0, 0.0);
    if (lead) {
        for (int k = 0; k < KP; ++k) {
            const double2 r = red[k * P + pp];
            sum.x += r.x;
            sum.y += r.y;
        }
    }
    if (I.n_ig > 1) {
        double2* part = reinterpret_cast<double2*>(A.part) + I.off_part;
        if (lead && colp_ok) part[task.ig * NP + pidx] = sum;
        if (!arrive_last(&A.counters[I.counter_off + task.cb], I.n_ig, &s_last)) return;
        sum = make_double2(0.0, 0.0);
        if (lead && colp_ok) {
            // the partial sums are requested PB item groups at a time and
            // added in item-group order: their loads overlap instead of
            // waiting for one another
            constexpr int PB = 8;
            for (int ig0 = 0; ig0 < I.n_ig; ig0 += PB) {
                double rx[PB], ry[PB];
#pragma unroll
                for (int k = 0; k < PB; ++k) {
                    rx[k] = ry[k] = 0.0;
                    if (ig0 + k < I.n_ig) {
                        const double* src = reinterpret_cast<const double*>(part + (ig0 + k) * NP + pidx);
                        rx[k] = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ry[k] = __hip_atomic_load(src + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
#pragma unroll
                for (int k = 0; k < PB; ++k) {
                    if (ig0 + k < I.n_ig) {
                        sum.x += rx[k];
                        sum.y += ry[k];
                    }
                }
            }
        }
        if (l == 0) A.counters[I.counter_off + task.cb] = 0u;
    }

    const double qs = I.q_scale;
    if constexpr (MODE == MODE_EVAL) {
        if (lead && colp_ok)
            reinterpret_cast<double2*>(A.out)[I.off_state + pidx] = make_double2(qs * sum.x, qs * sum.y);
    } else {
        cx<T>* nsb = reinterpret_cast<cx<T>*>(dyn + sizeof(double2) * KP * P);   // [N][GB]
        cx<T>* scr = nsb + P;                                                    // [slots][GB]
        if (lead) {
            double2 ns = make_double2(0.0, 0.0);
            if (colp_ok) {
                const double kx = qs * sum.x, ky = qs * sum.y, dt = A.dt;
                const long long idx = I.off_state + pidx;
                double2* yv = reinterpret_cast<double2*>(A.y);
                double2* ys = reinterpret_cast<double2*>(A.ystage);
                double2* ks = reinterpret_cast<double2*>(A.ksum);
                if (A.stage == 0) {
                    ks[idx] = make_double2(kx, ky);
                    ns = make_double2(yb.x + 0.5 * dt * kx, yb.y + 0.5 * dt * ky);
                    ys[idx] = ns;
                } else if (A.stage == 1 || A.stage == 2) {
                    ks[idx] = make_double2(kb.x + 2.0 * kx, kb.y + 2.0 * ky);
                    const double cst = A.stage == 1 ? 0.5 * dt : dt;
                    ns = make_double2(yb.x + cst * kx, yb.y + cst * ky);
                    ys[idx] = ns;
                } else {
                    ns = make_double2(yb.x + dt / 6.0 * (kb.x + kx), yb.y + dt / 6.0 * (kb.y + ky));
                    yv[idx] = ns;
                }
            }
            nsb[x * GB + pg] = to_t<T>(REAL ? make_double2(ns.x, 0.0) : ns);   // the real form evolves Re f
        }
        __syncthreads();
        // axis-0 forward transform of the next stage state, by the first block
        const bool b0 = bi == 0;
        cx<T> v[V];
#pragma unroll
        for (int m = 0; m < V; ++m) v[m] = b0 ? nsb[(t + TPT * m) * GB + g] : cx<T>{(T)0, (T)0};
        fft_dist<T, N, -1, WV, CPAD>(v, scr + g, GB, t, tw, b0);
        if (b0 && col_ok) {
            cx<T>* sp = reinterpret_cast<cx<T>*>(A.spec0) + I.off_spec0;
            const T sc = (T)I.fwd_scale;
            if constexpr (FUSED) {
#pragma unroll
                for (int m = 0; m < V; ++m) sp[(long long)c * N + t + TPT * m] = sc * v[m];
            } else {
#pragma unroll
                for (int m = 0; m < V; ++m) sp[(long long)(t + TPT * m) * C + c] = sc * v[m];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Fourier coefficients of a grid function, one axis per launch, in place, in
// double: the length-N forward DFT of every line along `axis`, times
// (-1)^i / N at output index i.  The grid starts at -L, so
// e^{-i pi j (-L + h x) / L} = (-1)^j e^{-2 pi i j x / N}; after all d axes
// the array holds g_hat_j = N^-d sum_x g(k_x) e^{-i pi j.k_x / L} in FFT
// index order, the coefficients of the series of eq. (fj).  GB lines per
// workgroup, neighbouring lines on neighbouring lanes; the twiddles are
// computed in the workgroup.
// ---------------------------------------------------------------------------
template <int N, int GB>
__global__ __launch_bounds__(GB* FftShape<N>::TPT) void k_axis_spectrum(double2* data, long long n_lines,
                                                                        long long stride) {
    using S = FftShape<N>;
    constexpr int TPT = S::TPT, V = S::V, PITCH = N + 1;
    __shared__ cx<double> lds[GB * PITCH];
    __shared__ cx<double> tw[N];
    const int l = threadIdx.x, g = l % GB, t = l / GB;
    for (int i = l; i < N; i += GB * TPT) {
        double sn, cs;
        sincospi(2.0 * i / N, &sn, &cs);
        tw[i] = cx<double>{cs, sn};
    }
    const long long line = (long long)blockIdx.x * GB + g;
    const bool active = line < n_lines;
    const long long outer = active ? line / stride : 0, inner = active ? line % stride : 0;
    double2* base = data + outer * N * stride + inner;
    cx<double> v[V];
#pragma unroll
    for (int m = 0; m < V; ++m) v[m] = active ? to_t<double>(base[(long long)(t + TPT * m) * stride]) : cx<double>{0.0, 0.0};
    __syncthreads();    // twiddles in LDS
    fft_dist<double, N, -1>(v, lds + g * PITCH, 1, t, tw, active);
    if (active) {
#pragma unroll
        for (int m = 0; m < V; ++m) {
            const int i = t + TPT * m;
            const double sc = (i & 1 ? -1.0 : 1.0) / N;
            base[(long long)i * stride] = make_double2(sc * v[m].x, sc * v[m].y);
        }
    }
}

// ---------------------------------------------------------------------------
// Plan tables: quadrature nodes, phase tables, unit weights, twiddles.  All
// in double on the GPU; float copies rounded once.
// ---------------------------------------------------------------------------
__global__ void k_nodes(const InstDev* insts, int idx, double* nodes) {
    const InstDev I = insts[idx];
    const int d = I.d;
    double* r = nodes + I.off_nodes;
    double* wr = r + I.Nr;
    double* qh = wr + I.Nr;
    double* ws = qh + I.Ns * d;
    double* sg = ws + I.Ns;
    double* wsig = sg + I.Nsig * d;
    const int nthr = blockDim.x;
    // Gauss-Legendre on [-1, 1] mapped to [0, R]
    const int n = I.Nr;
    for (int i = threadIdx.x; i < n; i += nthr) {
        double x, w;
        gl_root(n, i, &x, &w);
        r[n - 1 - i] = 0.5 * I.R * (1.0 + x);
        wr[n - 1 - i] = 0.5 * I.R * w;
    }
    // sphere rules, same rule for q-hat and sigma
    for (int which = 0; which < 2; ++which) {
        const int np = which == 0 ? I.Ns : I.Nsig;
        double* P = which == 0 ? qh : sg;
        double* Wt = which == 0 ? ws : wsig;
        for (int i = threadIdx.x; i < np; i += nthr) {
            if (d == 2) {
                double sn, cs;
                sincospi((2.0 * i + 1.0) / np, &sn, &cs);
                P[2 * i] = cs;
                P[2 * i + 1] = sn;
                Wt[i] = 2.0 * M_PI / np;
                continue;
            }
            double v[3] = {0.0, 0.0, 0.0};
            if (I.rule == 1) {                 // octahedron: +e0, -e0, +e1, ...
                v[i / 2] = (i & 1) ? -1.0 : 1.0;
            } else if (I.rule == 2) {          // cube: sign bits (4, 2, 1)
                const double q = 1.0 / sqrt(3.0);
                v[0] = (i & 4) ? -q : q;
                v[1] = (i & 2) ? -q : q;
                v[2] = (i & 1) ? -q : q;
            } else {                           // icosahedron: cyclic (0, +-1, +-phi)
                const double phi = 0.5 * (1.0 + sqrt(5.0));
                const double nr = sqrt(1.0 + phi * phi);
                const int cyc = i / 4, s1 = (i >> 1) & 1, s2 = i & 1;
                const double u[3] = {0.0, s1 ? -1.0 : 1.0, s2 ? -phi : phi};
                for (int a = 0; a < 3; ++a) v[(a + cyc) % 3] = u[a] / nr;
            }
            for (int a = 0; a < 3; ++a) P[3 * i + a] = v[a];
            Wt[i] = 4.0 * M_PI / np;
        }
    }
}

__global__ void k_phase(const InstDev* insts, int idx, const double* nodes, double2* ph64, float2* ph32) {
    const InstDev I = insts[idx];
    const int d = I.d, N = I.N;
    // the real form adds one row, shift n_shift = the zero vector (the
    // unshifted field), and drops the Nyquist index j = -N/2 of every row
    const long long total = (long long)(I.n_shift + I.nyq_zero) * d * N;
    const double* r = nodes + I.off_nodes;
    const double* qh = r + 2 * I.Nr;
    const double* sg = qh + I.Ns * (d + 1);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int ls = (int)(e / (d * N));
        const int rem = (int)(e % (d * N));
        const int a = rem / N, i = rem % N;
        double s = 0.0;
        if (ls < I.n_shift) {
            const int it = ls / I.S_item, k = ls % I.S_item;
            const int p1 = it / I.Ns, p2 = it % I.Ns;
            const double rr = r[p1], q = qh[p2 * d + a];
            if (k == 0) s = rr * q;                                       // s_a = r q-hat
            else if (k <= I.Nsig) s = 0.5 * rr * (q - sg[(k - 1) * d + a]);   // s_b
            else s = 0.5 * rr * (q + sg[(k - 1 - I.Nsig) * d + a]);         // s_c
        }
        const int j = i < N / 2 ? i : i - N;
        double sn, cs;
        sincospi((double)j * s / I.L, &sn, &cs);
        double2 v = make_double2(cs, -sn);                            // exp(-i pi j s / L)
        if (I.nyq_zero && i == N / 2) v = make_double2(0.0, 0.0);
        ph64[I.off_ph + e] = v;
        if (ph32) ph32[I.off_ph + e] = make_float2((float)v.x, (float)v.y);
    }
}

__global__ void k_unitw(const InstDev* insts, int idx, const double* nodes, const UnitPat* pat,
                        double* uw64, float* uw32) {
    const InstDev I = insts[idx];
    const int d = I.d;
    const double* r = nodes + I.off_nodes;
    const double* wr = r + I.Nr;
    const double* ws = wr + I.Nr + I.Ns * d;
    const double* wsig = ws + I.Ns + I.Nsig * d;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < I.n_unit; e += gridDim.x * blockDim.x) {
        const int it = e / I.U_item, u = e % I.U_item;
        const int p1 = it / I.Ns, p2 = it % I.Ns;
        const UnitPat p = pat[u];
        double rp = 1.0;
        for (int k = 0; k < 2 * d - 3; ++k) rp *= r[p1];              // |q|^(2d-3)
        double wsg = wsig[p.p3] + (p.p3b >= 0 ? wsig[p.p3b] : 0.0);
        const double W = wr[p1] * rp * ws[p2] * wsg;
        uw64[I.off_unit + e] = W;
        if (uw32) uw32[I.off_unit + e] = (float)W;
    }
}

// Axis-1 interpolation kernel of each slab field (2D): K_h(y) = sum over j1
// of ph_h(j1) e^{+2 pi i j1 y / N}, ph_h the axis-1 phase row of the slab
// field's representative shift.  In double; the float copy rounded once.
__global__ void k_ktab(const InstDev* insts, int idx, const double2* ph64, const int* hrep, double2* kt64,
                       float2* kt32) {
    const InstDev I = insts[idx];
    const int N = I.N;
    // each row twice over, [slab field][2N], so that a run of x values reads
    // K_h(c - x) without a wrap
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < I.n_slab * 2 * N; e += gridDim.x * blockDim.x) {
        const int h = e / (2 * N), y = e % N;
        const double2* row = ph64 + I.off_ph + (long long)hrep[I.off_hrep + h] * 2 * N + N;
        double sx = 0.0, sy = 0.0;
        for (int j1 = 0; j1 < N; ++j1) {
            double sn, cs;
            sincospi(2.0 * (double)((j1 * y) % N) / N, &sn, &cs);
            const double2 p = row[j1];
            sx += p.x * cs - p.y * sn;
            sy += p.x * sn + p.y * cs;
        }
        kt64[I.off_kt + e] = make_double2(sx, sy);
        if (kt32) kt32[I.off_kt + e] = make_float2((float)sx, (float)sy);
    }
}

__global__ void k_twiddles(int N, double2* tw64, float2* tw32) {
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * k / N, &sn, &cs);
        tw64[k] = make_double2(cs, sn);
        tw32[k] = make_float2((float)cs, (float)sn);
    }
}

// ---------------------------------------------------------------------------
// Moments: one workgroup per instance, fixed-order tree reduction.
// ---------------------------------------------------------------------------
// The lane's share of the moment sums over an instance of dimension DD
// (a compile-time dimension keeps every per-axis array in registers).
template <int DD>
__device__ __forceinline__ void moment_sums(const InstDev& I, const double2* f, double (&acc)[6], double& bad) {
    const int N = I.N;
    // the grid index of the lane's point as base-N digits (last axis
    // fastest), advanced by the workgroup size with carries: no integer
    // division inside the loop (a 64-bit one is a long software routine)
    int dig[DD], step[DD];
    {
        unsigned rx = threadIdx.x, rs = blockDim.x;
#pragma unroll
        for (int a = DD - 1; a >= 0; --a) {
            dig[a] = (int)(rx % (unsigned)N);
            step[a] = (int)(rs % (unsigned)N);
            rx /= (unsigned)N;
            rs /= (unsigned)N;
        }
        dig[0] += (int)rx * N;      // whatever the top digit overflows stays in it
        step[0] += (int)rs * N;
    }
    // eight of the lane's points requested at a time, then added in order
    constexpr int PB = 8;
    const long long stride = blockDim.x;
    for (long long x0 = threadIdx.x; x0 < I.n_pts; x0 += PB * stride) {
        double2 vb[PB];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const long long x = x0 + b * stride;
            vb[b] = x < I.n_pts ? f[x] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            if (x0 + b * stride >= I.n_pts) break;
            const double2 v = vb[b];
            double k[DD], k2 = 0;
#pragma unroll
            for (int a = DD - 1; a >= 0; --a) {
                k[a] = -I.L + I.h * (double)dig[a];
                k2 += k[a] * k[a];
            }
            int carry = 0;
#pragma unroll
            for (int a = DD - 1; a >= 1; --a) {
                dig[a] += step[a] + carry;
                carry = dig[a] >= N ? 1 : 0;
                if (carry) dig[a] -= N;
            }
            dig[0] += step[0] + carry;
            acc[0] += v.x;
            acc[1] += v.x * k2;
#pragma unroll
            for (int a = 0; a < DD; ++a) acc[2 + a] += v.x * k[a];
            acc[5] = fmax(acc[5], fabs(v.y));
            if (!isfinite(v.x) || !isfinite(v.y)) bad = 1.0;
        }
    }
}

__global__ __launch_bounds__(1024) void k_moments(const InstDev* insts, const double* f_, double* out) {
    const InstDev& I = insts[blockIdx.x];
    const double2* f = reinterpret_cast<const double2*>(f_) + I.off_state;
    const int d = I.d;
    double acc[6] = {0, 0, 0, 0, 0, 0};   // rho, E, P0, P1, P2, max|Im|
    double bad = 0.0;
    if (d == 3)
        moment_sums<3>(I, f, acc, bad);
    else
        moment_sums<2>(I, f, acc, bad);
    __shared__ double red[7][1024];
    for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = acc[q];
    red[6][threadIdx.x] = bad;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int q = 0; q < 5; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
            red[5][threadIdx.x] = fmax(red[5][threadIdx.x], red[5][threadIdx.x + w]);
            red[6][threadIdx.x] = fmax(red[6][threadIdx.x], red[6][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double hd = 1.0;
        for (int a = 0; a < d; ++a) hd *= I.h;
        double* o = out + 7 * blockIdx.x;
        for (int q = 0; q < 5; ++q) o[q] = hd * red[q][0];
        o[5] = red[5][0];
        o[6] = red[6][0];
    }
}

// ---------------------------------------------------------------------------
// Trigonometric resampling between the grids of N and P = 2N points per axis
// (both span [-L, L) from -L).  With g(m) = sum_{j=-N/2}^{N/2-1} e^{2 pi i j m / P},
// which vanishes for even m != 0 (mod P) and equals N at m = 0, and the
// kernel h_k = g(2k + 1), k = 0..N-1:
//   refining (the truncated series f_N evaluated on the fine grid, eq. (fj)):
//     u_{2q} = v_q,   u_{2q+1} = (1/N) sum_x h_{(q-x) mod N} v_x;
//   coarsening (projection of a fine-grid function onto the modes
//   [-N/2, N/2-1], sampled on the coarse grid):
//     w_q = u_{2q} / 2 + (1/P) sum_s h_{(q-1-s) mod N} u_{2s+1};
//   projecting (the same projection, kept on the fine grid):
//     w_{2q} as above,   w_{2q+1} = u_{2q+1} / 2 + (1/P) sum_s h_{(q-s) mod N} u_{2s}.
// A workgroup takes `lt` consecutive lines along the resampled axis (a line
// is fixed by the indices of the other axes), stages them and the kernel
// (twice over, so that the index (k0 - s) mod N needs no wrap) in LDS, and
// computes from there, one thread per (line, q): the pair of fine points
// 2q, 2q+1 (refining, projecting) or the coarse point q (coarsening).  N is a
// multiple of 4 and the N-term sums run as four interleaved partial sums.
// Lines are coalesced along the line when the axis is the fastest one
// (inner == 1), else across lines.  grid.y runs over instances.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 rs_sum(const double2* hh, int kb, const double2* xs, int xstride, int N) {
    double re[4] = {0.0, 0.0, 0.0, 0.0}, im[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < N; s += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double2 c = hh[kb - s - u], v = xs[(s + u) * xstride];
            re[u] += c.x * v.x - c.y * v.y;
            im[u] += c.x * v.y + c.y * v.x;
        }
    }
    return make_double2((re[0] + re[1]) + (re[2] + re[3]), (im[0] + im[1]) + (im[2] + im[3]));
}

// Classical RK4 stage update at one point: stage 0..2 write the stage state
// ys and the derivative sum ks, stage 3 the new state y.
__device__ __forceinline__ double2 rk_stage(const RkStage& e, long long i, double2 k) {
    double2* y = reinterpret_cast<double2*>(e.y);
    double2* ys = reinterpret_cast<double2*>(e.ys);
    double2* ks = reinterpret_cast<double2*>(e.ks);
    const double dt = e.dt;
    const double2 y0 = y[i];
    double2 ns;
    if (e.stage == 0) {
        ks[i] = k;
        ns = make_double2(y0.x + 0.5 * dt * k.x, y0.y + 0.5 * dt * k.y);
        ys[i] = ns;
    } else if (e.stage == 1 || e.stage == 2) {
        const double2 k0 = ks[i];
        const double cst = e.stage == 1 ? 0.5 * dt : dt;
        ks[i] = make_double2(k0.x + 2.0 * k.x, k0.y + 2.0 * k.y);
        ns = make_double2(y0.x + cst * k.x, y0.y + cst * k.y);
        ys[i] = ns;
    } else {
        const double2 k0 = ks[i];
        ns = make_double2(y0.x + dt / 6.0 * (k0.x + k.x), y0.y + dt / 6.0 * (k0.y + k.y));
        y[i] = ns;
    }
    return ns;
}

template <int KIND>
__global__ __launch_bounds__(256) void k_resample(const ResampleDesc* rd, const double2* htab,
                                                  const double2* in, double2* out, int lt) {
    extern __shared__ double2 rs_smem[];
    const ResampleDesc D = rd[blockIdx.y];
    const int m_in = D.m_in, m_out = D.m_out, N = D.N;
    const long long inner = D.inner;
    const long long n_lines = D.n_out / m_out;
    const long long L0 = (long long)blockIdx.x * lt;
    if (L0 >= n_lines) return;
    const int nl = (int)min((long long)lt, n_lines - L0);
    double2* hh = rs_smem;                     // h_{i mod N}, i < 2N
    double2* xt = rs_smem + 2 * N;             // [m_in][lt]
    for (int i = threadIdx.x; i < 2 * N; i += 256) hh[i] = htab[D.h_off + (i < N ? i : i - N)];
    const double2* src = in + D.in_off;
    for (int i = threadIdx.x; i < nl * m_in; i += 256) {
        const int l = inner == 1 ? i / m_in : i % nl;
        const int s = inner == 1 ? i % m_in : i / nl;
        const long long L = L0 + l;
        xt[s * lt + l] = src[(L / inner) * m_in * inner + s * inner + L % inner];
    }
    __syncthreads();
    const double inv_p = 1.0 / (2 * N);
    for (int i = threadIdx.x; i < nl * N; i += 256) {
        const int l = inner == 1 ? i / N : i % nl;
        const int q = inner == 1 ? i % N : i / nl;
        const long long L = L0 + l;
        const long long base = D.out_off + (L / inner) * m_out * inner + L % inner;
        const double2* xl = xt + l;
        if constexpr (KIND == RS_REFINE) {
            const double2 sm = rs_sum(hh, q + N, xl, lt, N);
            out[base + (long long)(2 * q) * inner] = xl[q * lt];
            out[base + (long long)(2 * q + 1) * inner] = make_double2(sm.x / N, sm.y / N);
        } else {
            // even fine point (or coarse point q) from the odd fine points
            const double2 se = rs_sum(hh, q - 1 + N, xl + lt, 2 * lt, N);
            const double2 ve = xl[(2 * q) * lt];
            const double2 we = make_double2(0.5 * ve.x + se.x * inv_p, 0.5 * ve.y + se.y * inv_p);
            if constexpr (KIND == RS_COARSEN) {
                out[base + (long long)q * inner] = we;
            } else {
                const double2 so = rs_sum(hh, q + N, xl, 2 * lt, N);
                const double2 vo = xl[(2 * q + 1) * lt];
                out[base + (long long)(2 * q) * inner] = we;
                out[base + (long long)(2 * q + 1) * inner] =
                    make_double2(0.5 * vo.x + so.x * inv_p, 0.5 * vo.y + so.y * inv_p);
            }
        }
    }
}

// Even fine-grid samples of a fine-grid function onto the coarse grid (exact
// for functions of the modes [-N/2, N/2-1]).  rd: the coarsening descriptors
// of the last axis (their out_off is the coarse packing); in_off of the
// instance's fine data comes from fine_off.
__global__ __launch_bounds__(256) void k_decimate(const ResampleDesc* rd, const long long* fine_off, int d,
                                                  const double2* in, double2* out) {
    const ResampleDesc D = rd[blockIdx.y];
    const int N = D.N, P = 2 * N;
    long long np = 1;
    for (int a = 0; a < d; ++a) np *= N;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= np) return;
    long long rem = t, fi = 0, st = 1;
    for (int a = d - 1; a >= 0; --a) {
        fi += 2 * (rem % N) * st;
        rem /= N;
        st *= P;
    }
    out[D.out_off + t] = in[fine_off[blockIdx.y] + fi];
}

// ---------------------------------------------------------------------------
// Exact-Galerkin RK4 stage on the fine grid (P points per axis, the
// template's N), one column (axis 0) per group of lanes: the column of Q,
// already projected onto the coarse modes along the other axes, is
// transformed along axis 0 (double), its modes outside [-P/4, P/4-1] are
// dropped and it is transformed back: that is Q projected onto the modes of
// the coarse grid.  Then the classical RK4 stage update of the fine-grid
// state, and the axis-0 forward transform of the new stage state into spec0
// (in T), as the column forward transform stores it.
// ---------------------------------------------------------------------------
template <class T, int D, int N, int GB>
__global__ __launch_bounds__(GB* FftShape<N>::TPT) void k_colrk(ColRkArgs A) {
    using S = FftShape<N>;
    constexpr int TPT = S::TPT, V = S::V, PITCH = N + 1;
    constexpr int C = (int)ipow_c(N, D - 1);
    __shared__ cx<double> lds64[GB * PITCH];
    __shared__ cx<double> tw64[N];
    __shared__ cx<T> ldsT[sizeof(T) == 8 ? 1 : GB * PITCH];
    __shared__ cx<T> twT[sizeof(T) == 8 ? 1 : N];
    const TaskB task = A.tasks[xcd_task(blockIdx.x, gridDim.x)];
    const InstDev& I = A.inst[task.inst];
    const int l = threadIdx.x, g = l % GB, t = l / GB;
    const int c = task.cb * GB + g;
    const bool active = c < C;
    const cx<double>* twg64 = reinterpret_cast<const cx<double>*>(A.tw64) + I.off_tw;
    for (int i = l; i < N; i += GB * TPT) tw64[i] = twg64[i];
    if constexpr (sizeof(T) != 8) {
        const cx<T>* twg = reinterpret_cast<const cx<T>*>(A.tw) + I.off_tw;
        for (int i = l; i < N; i += GB * TPT) twT[i] = twg[i];
    }
    __syncthreads();
    const long long off = I.off_state;
    const double2* q = reinterpret_cast<const double2*>(A.q) + off;
    cx<double> v[V];
#pragma unroll
    for (int m = 0; m < V; ++m) {
        const double2 x = active ? q[(long long)(t + TPT * m) * C + c] : make_double2(0.0, 0.0);
        v[m] = cx<double>{x.x, x.y};
    }
    fft_dist<double, N, -1>(v, lds64 + g * PITCH, 1, t, tw64, active);
#pragma unroll
    for (int m = 0; m < V; ++m) {
        const int i = t + TPT * m;
        if (i >= N / 4 && i < N - N / 4) v[m] = cx<double>{0.0, 0.0};
    }
    fft_dist<double, N, 1>(v, lds64 + g * PITCH, 1, t, tw64, active);
    RkStage e{A.stage, A.dt, A.y + 2 * off, A.ys + 2 * off, A.ks + 2 * off};
    cx<T> nx[V];
    const double inv = 1.0 / N;
#pragma unroll
    for (int m = 0; m < V; ++m) {
        nx[m] = cx<T>{(T)0, (T)0};
        if (!active) continue;
        const double2 ns = rk_stage(e, (long long)(t + TPT * m) * C + c, make_double2(inv * v[m].x, inv * v[m].y));
        nx[m] = to_t<T>(ns);
    }
    if constexpr (sizeof(T) == 8) {
        fft_dist<T, N, -1>(nx, reinterpret_cast<cx<T>*>(lds64) + g * PITCH, 1, t,
                           reinterpret_cast<const cx<T>*>(tw64), active);
    } else {
        fft_dist<T, N, -1>(nx, ldsT + g * PITCH, 1, t, twT, active);
    }
    cx<T>* sp = reinterpret_cast<cx<T>*>(A.spec0) + I.off_spec0;
    const T sc = (T)I.fwd_scale;
    if (active) {
        if (D == 2 && A.spec_trans) {
#pragma unroll
            for (int m = 0; m < V; ++m) sp[(long long)c * N + t + TPT * m] = sc * nx[m];
        } else {
#pragma unroll
            for (int m = 0; m < V; ++m) sp[(long long)(t + TPT * m) * C + c] = sc * nx[m];
        }
    }
}

// ---------------------------------------------------------------------------
// Template geometry and dispatch.
// ---------------------------------------------------------------------------
template <class T, int D, int N> constexpr int igs_of() {
    return sizeof(T) == 8 ? Geo<D, N>::IGS64 : Geo<D, N>::IGS32;
}

// Launch with or without start/stop events bound to the dispatch itself
// (the events then bracket exactly the kernel's execution).
#define WKE_LAUNCH(KERNEL, GRID, BLOCK, STREAM, EV, ...)                                           \
    do {                                                                                           \
        if ((EV) && (EV)->start)                                                                   \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, (EV)->start, (EV)->stop, 0, __VA_ARGS__); \
        else                                                                                       \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, __VA_ARGS__);                       \
    } while (0)

template <class T, int D, int N> static hipError_t go_colfwd(const ColFwdArgs& a, int ntasks, hipStream_t s,
                                                             const LaunchEvents*) {
    constexpr int GF = Geo<D, N>::GF;
    hipLaunchKernelGGL((k_colfwd<T, D, N, GF>), dim3(ntasks), dim3(GF * Geo<D, N>::TPT), 0, s, a);
    return hipGetLastError();
}
template <class T, int D, int N> static hipError_t go_colrk(const ColRkArgs& a, int ntasks, hipStream_t s,
                                                            const LaunchEvents*) {
    constexpr int GF = Geo<D, N>::GF;
    hipLaunchKernelGGL((k_colrk<T, D, N, GF>), dim3(ntasks), dim3(GF * Geo<D, N>::TPT), 0, s, a);
    return hipGetLastError();
}
template <class T, int D, int N> static hipError_t go_passA(const PassAArgs& a, int ntasks, hipStream_t s,
                                                            const LaunchEvents* ev) {
    if constexpr (D == 2) {
        constexpr int JB = sizeof(T) == 8 ? Geo<D, N>::JB64 : Geo<D, N>::JB32;
        constexpr int SB = sizeof(T) == 8 ? Geo<D, N>::SB64 : Geo<D, N>::SB32;
        WKE_LAUNCH((k_passA2d<T, N, JB, SB>), dim3(ntasks), dim3(JB * SB * Geo<D, N>::TPT), s, ev, a);
    } else {
        if constexpr (sizeof(T) == 8 ? Geo<D, N>::REG3_64 : Geo<D, N>::REG3_32) {
            constexpr int NW = sizeof(T) == 8 ? Geo<D, N>::NWR64 : Geo<D, N>::NWR32;
            WKE_LAUNCH((k_passA3d_reg<T, N, NW>), dim3(ntasks), dim3(64 * NW), s, ev, a);
        } else {
            constexpr int GA = Geo<D, N>::GA3;
            constexpr int SC = sizeof(T) == 8 ? Geo<D, N>::SC64 : Geo<D, N>::SC32;
            constexpr int SCA = sizeof(T) == 8 ? Geo<D, N>::SC64_ALT : 0;
            if constexpr (SCA > 0) {
                if (a.slab_alt) {
                    WKE_LAUNCH((k_passA3d<T, N, GA, SCA>), dim3(ntasks), dim3(GA * Geo<D, N>::TPT * SCA), s, ev, a);
                    return hipGetLastError();
                }
            }
            if (a.slab_alt) return hipErrorInvalidValue;
            WKE_LAUNCH((k_passA3d<T, N, GA, SC>), dim3(ntasks), dim3(GA * Geo<D, N>::TPT * SC), s, ev, a);
        }
    }
    return hipGetLastError();
}
template <class T, int D, int N, int MODE, int FUS, bool REAL, bool ONE>
static hipError_t go_passB_fp1(const PassBArgs& a, int ntasks, hipStream_t s, const LaunchEvents* ev) {
    constexpr bool FUSED = FUS != 0;
    static const hipError_t attr =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_passB_fp<T, D, N, MODE, FUS, REAL, ONE>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)FP_LDS_LIMIT);
    if (attr != hipSuccess) return attr;
    if (a.fp_lds > FP_LDS_LIMIT || a.fp_threads > fp_max_threads(sizeof(T) == 8 ? 0 : 1, N, FUSED, REAL) ||
        a.fp_threads <= 0 || a.fp_threads % 64)
        return hipErrorInvalidValue;
    if (ev && ev->start)
        hipExtLaunchKernelGGL((k_passB_fp<T, D, N, MODE, FUS, REAL, ONE>), dim3(ntasks), dim3(a.fp_threads), a.fp_lds, s,
                              ev->start, ev->stop, 0, a);
    else
        hipLaunchKernelGGL((k_passB_fp<T, D, N, MODE, FUS, REAL, ONE>), dim3(ntasks), dim3(a.fp_threads), a.fp_lds, s,
                           a);
    return hipGetLastError();
}
template <class T, int D, int N, int MODE, int FUS>
static hipError_t go_passB_fp(const PassBArgs& a, int ntasks, hipStream_t s, const LaunchEvents* ev) {
    if constexpr (FUS != 0) {
        if (a.one)
            return a.real ? go_passB_fp1<T, D, N, MODE, FUS, true, true>(a, ntasks, s, ev)
                          : go_passB_fp1<T, D, N, MODE, FUS, false, true>(a, ntasks, s, ev);
    }
    return a.real ? go_passB_fp1<T, D, N, MODE, FUS, true, false>(a, ntasks, s, ev)
                  : go_passB_fp1<T, D, N, MODE, FUS, false, false>(a, ntasks, s, ev);
}
template <class T, int D, int N> static hipError_t go_passB(const PassBArgs& a, int ntasks, hipStream_t s,
                                                            const LaunchEvents* ev) {
    if (a.fp_threads > 0) {
        if constexpr (D == 2) {
            if (a.fp_fused && a.fp_mfma)
                return a.mode == MODE_RK ? go_passB_fp<T, D, N, MODE_RK, 2>(a, ntasks, s, ev)
                                         : go_passB_fp<T, D, N, MODE_EVAL, 2>(a, ntasks, s, ev);
            if (a.fp_fused)
                return a.mode == MODE_RK ? go_passB_fp<T, D, N, MODE_RK, 1>(a, ntasks, s, ev)
                                         : go_passB_fp<T, D, N, MODE_EVAL, 1>(a, ntasks, s, ev);
        }
        return a.mode == MODE_RK ? go_passB_fp<T, D, N, MODE_RK, 0>(a, ntasks, s, ev)
                                 : go_passB_fp<T, D, N, MODE_EVAL, 0>(a, ntasks, s, ev);
    }
    if (a.real) return hipErrorInvalidValue;     // the real form has no item-slot kernel
    constexpr int GB = Geo<D, N>::GB, IGS = igs_of<T, D, N>();
    if (a.mode == MODE_RK)
        WKE_LAUNCH((k_passB<T, D, N, GB, IGS, MODE_RK>), dim3(ntasks), dim3(GB * Geo<D, N>::TPT * IGS), s, ev, a);
    else
        WKE_LAUNCH((k_passB<T, D, N, GB, IGS, MODE_EVAL>), dim3(ntasks), dim3(GB * Geo<D, N>::TPT * IGS), s, ev, a);
    return hipGetLastError();
}

#define WKE_DISPATCH(FN, ARGS)                                                         \
    do {                                                                               \
        if (ntasks <= 0) return hipSuccess;                                            \
        if (prec == 0) {                                                               \
            if (d == 2) {                                                              \
                switch (N) {                                                           \
                    case 16: return FN<double, 2, 16>(ARGS, ntasks, s, ev);                \
                    case 32: return FN<double, 2, 32>(ARGS, ntasks, s, ev);                \
                    case 48: return FN<double, 2, 48>(ARGS, ntasks, s, ev);                \
                    case 64: return FN<double, 2, 64>(ARGS, ntasks, s, ev);                \
                    case 96: return FN<double, 2, 96>(ARGS, ntasks, s, ev);                \
                    case 128: return FN<double, 2, 128>(ARGS, ntasks, s, ev);              \
                }                                                                      \
            } else {                                                                   \
                switch (N) {                                                           \
                    case 16: return FN<double, 3, 16>(ARGS, ntasks, s, ev);                \
                    case 32: return FN<double, 3, 32>(ARGS, ntasks, s, ev);                \
                    case 64: return FN<double, 3, 64>(ARGS, ntasks, s, ev);                \
                }                                                                      \
            }                                                                          \
        } else {                                                                       \
            if (d == 2) {                                                              \
                switch (N) {                                                           \
                    case 16: return FN<float, 2, 16>(ARGS, ntasks, s, ev);                 \
                    case 32: return FN<float, 2, 32>(ARGS, ntasks, s, ev);                 \
                    case 48: return FN<float, 2, 48>(ARGS, ntasks, s, ev);                 \
                    case 64: return FN<float, 2, 64>(ARGS, ntasks, s, ev);                 \
                    case 96: return FN<float, 2, 96>(ARGS, ntasks, s, ev);                 \
                    case 128: return FN<float, 2, 128>(ARGS, ntasks, s, ev);               \
                }                                                                      \
            } else {                                                                   \
                switch (N) {                                                           \
                    case 16: return FN<float, 3, 16>(ARGS, ntasks, s, ev);                 \
                    case 32: return FN<float, 3, 32>(ARGS, ntasks, s, ev);                 \
                    case 64: return FN<float, 3, 64>(ARGS, ntasks, s, ev);                 \
                }                                                                      \
            }                                                                          \
        }                                                                              \
        return hipErrorInvalidValue;                                                   \
    } while (0)

hipError_t launch_colfwd(int prec, int d, int N, const ColFwdArgs& a, int ntasks, hipStream_t s) {
    const LaunchEvents* ev = nullptr;
    WKE_DISPATCH(go_colfwd, a);
}
hipError_t launch_colrk(int prec, int d, int N, const ColRkArgs& a, int ntasks, hipStream_t s) {
    const LaunchEvents* ev = nullptr;
    WKE_DISPATCH(go_colrk, a);
}
hipError_t launch_passA(int prec, int d, int N, const PassAArgs& a, int ntasks, hipStream_t s,
                        const LaunchEvents* ev) {
    WKE_DISPATCH(go_passA, a);
}
hipError_t launch_passB(int prec, int d, int N, const PassBArgs& a, int ntasks, hipStream_t s,
                        const LaunchEvents* ev) {
    WKE_DISPATCH(go_passB, a);
}

template <int N> static hipError_t go_spectrum(double* data, int d, int axis, hipStream_t s) {
    constexpr int GB = 8;
    long long lines = 1, stride = 1;
    for (int a = 0; a < d - 1; ++a) lines *= N;
    for (int a = axis + 1; a < d; ++a) stride *= N;
    const long long blocks = (lines + GB - 1) / GB;
    hipLaunchKernelGGL((k_axis_spectrum<N, GB>), dim3((unsigned)blocks), dim3(GB * FftShape<N>::TPT), 0, s,
                       reinterpret_cast<double2*>(data), lines, stride);
    return hipGetLastError();
}

hipError_t launch_spectrum(int d, int N, double* data, hipStream_t s) {
    if (d < 2 || d > 3) return hipErrorInvalidValue;
    for (int axis = 0; axis < d; ++axis) {
        hipError_t e;
        switch (N) {
            case 8: e = go_spectrum<8>(data, d, axis, s); break;
            case 16: e = go_spectrum<16>(data, d, axis, s); break;
            case 32: e = go_spectrum<32>(data, d, axis, s); break;
            case 48: e = go_spectrum<48>(data, d, axis, s); break;
            case 64: e = go_spectrum<64>(data, d, axis, s); break;
            case 96: e = go_spectrum<96>(data, d, axis, s); break;
            case 128: e = go_spectrum<128>(data, d, axis, s); break;
            default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_tables(const InstDev* inst_dev, const InstDev& I, int idx, double* nodes,
                         const UnitPat* upat_dev, double* ph64, float* ph32, double* uw64, float* uw32,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_nodes, dim3(1), dim3(256), 0, s, inst_dev, idx, nodes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long total = (long long)I.n_shift * I.d * I.N;
    const int blocks = (int)((total + 255) / 256 > 4096 ? 4096 : (total + 255) / 256);
    hipLaunchKernelGGL(k_phase, dim3(blocks), dim3(256), 0, s, inst_dev, idx, (const double*)nodes,
                       reinterpret_cast<double2*>(ph64), reinterpret_cast<float2*>(ph32));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_unitw, dim3((I.n_unit + 255) / 256), dim3(256), 0, s, inst_dev, idx,
                       (const double*)nodes, upat_dev, uw64, uw32);
    return hipGetLastError();
}

hipError_t launch_ktab(const InstDev* inst_dev, const InstDev& I, int idx, const double* ph64, const int* hrep,
                       double* kt64, float* kt32, hipStream_t s) {
    const int total = I.n_slab * 2 * I.N;
    if (I.d != 2 || total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ktab, dim3((total + 255) / 256), dim3(256), 0, s, inst_dev, idx,
                       reinterpret_cast<const double2*>(ph64), hrep, reinterpret_cast<double2*>(kt64),
                       reinterpret_cast<float2*>(kt32));
    return hipGetLastError();
}

hipError_t launch_twiddles(int N, double* tw64, float* tw32, hipStream_t s) {
    hipLaunchKernelGGL(k_twiddles, dim3(1), dim3(128), 0, s, N, reinterpret_cast<double2*>(tw64),
                       reinterpret_cast<float2*>(tw32));
    return hipGetLastError();
}

hipError_t launch_moments(const InstDev* inst, int batch, const double* f, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_moments, dim3(batch), dim3(1024), 0, s, inst, f, out);
    return hipGetLastError();
}

hipError_t launch_resample(int kind, const ResampleDesc* rd, int batch, const ResampleLaunch& g, const double* h,
                           const double* in, double* out, hipStream_t s) {
    if (batch < 1 || batch > 65535 || g.blocks < 1 || g.lt < 1 || g.lds > 64 * 1024) return hipErrorInvalidValue;
    const dim3 grid((unsigned)g.blocks, (unsigned)batch);
    const double2* h2 = reinterpret_cast<const double2*>(h);
    const double2* in2 = reinterpret_cast<const double2*>(in);
    double2* out2 = reinterpret_cast<double2*>(out);
    if (kind == RS_REFINE)
        hipLaunchKernelGGL((k_resample<RS_REFINE>), grid, dim3(256), g.lds, s, rd, h2, in2, out2, g.lt);
    else if (kind == RS_PROJECT)
        hipLaunchKernelGGL((k_resample<RS_PROJECT>), grid, dim3(256), g.lds, s, rd, h2, in2, out2, g.lt);
    else
        hipLaunchKernelGGL((k_resample<RS_COARSEN>), grid, dim3(256), g.lds, s, rd, h2, in2, out2, g.lt);
    return hipGetLastError();
}

hipError_t launch_decimate(const ResampleDesc* rd, const long long* fine_off, int batch, int d, int n_max,
                           const double* in, double* out, hipStream_t s) {
    long long np = 1;
    for (int a = 0; a < d; ++a) np *= n_max;
    if (batch < 1 || batch > 65535 || np < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_decimate, dim3((unsigned)((np + 255) / 256), (unsigned)batch), dim3(256), 0, s, rd,
                       fine_off, d, reinterpret_cast<const double2*>(in), reinterpret_cast<double2*>(out));
    return hipGetLastError();
}

}  // namespace wke
