// Compile-time shapes of the transforms and launch geometry of the kernel
// template instances: plain C++ (no HIP), shared by the kernels and by the
// host-side plan layout.
#pragma once

namespace wke {

constexpr long long ipow_c(int b, int e) { return e == 0 ? 1 : b * ipow_c(b, e - 1); }


// ---------------------------------------------------------------------------
// Radix plans.  The first radix must divide the last one (so the first
// stage can read the lane-distributed registers directly).
// ---------------------------------------------------------------------------
template <int... Rs> struct Radices {};

template <int N> struct PlanOf;
template <> struct PlanOf<8>   { using type = Radices<8>; };
template <> struct PlanOf<16>  { using type = Radices<4, 4>; };
template <> struct PlanOf<32>  { using type = Radices<4, 8>; };
template <> struct PlanOf<48>  { using type = Radices<4, 12>; };
template <> struct PlanOf<64>  { using type = Radices<8, 8>; };
template <> struct PlanOf<96>  { using type = Radices<4, 3, 8>; };
template <> struct PlanOf<128> { using type = Radices<4, 4, 8>; };

template <class P> struct PlanInfo;
template <int R0, int... Rs> struct PlanInfo<Radices<R0, Rs...>> {
    static constexpr int first = R0;
    static constexpr int count = 1 + sizeof...(Rs);
    static constexpr int last = [] {
        int a[] = {R0, Rs...};
        return a[sizeof...(Rs)];
    }();
};

template <int N> struct FftShape {
    using P = typename PlanOf<N>::type;
    static constexpr int R0 = PlanInfo<P>::first;
    static constexpr int RL = PlanInfo<P>::last;
    static constexpr int NST = PlanInfo<P>::count;
    static constexpr int TPT = N / RL;   // lanes per transform
    static constexpr int V = RL;         // values per lane
    static_assert(RL % R0 == 0, "first radix must divide the last");
};

// Padding pays where the first radix is 8 (lanes 8 elements apart: every
// lane of a transform on the same banks); with a first radix of 4 the
// conflicts are 2-way at most and the larger scratch costs more than it
// saves.  pad_scratch is the pad step (0: none) of a transform's LDS
// scratch and scratch_slots its size: N + N / 8 when padded (the last
// element sits at N - 1 + (N - 1) / 8), which also makes neighbouring
// transforms' scratch start 64 bytes apart in float, on the other half of
// the 128-byte bank cycle.
template <int N> constexpr int pad_scratch() { return FftShape<N>::R0 == 8 ? 8 : 0; }
template <int N> constexpr int scratch_slots() { return pad_scratch<N>() ? N + N / 8 : N + 1; }
// The field-parallel column pass (which in 3D interleaves the scratch of a
// field block's 4 columns element by element) uses the same padding.  A
// spare slot every R0 = 4 elements at N = 32 would also clear the first
// stage's remaining bank conflicts there (the 32-bank count, confirmed by
// the counters: 17-25% of LDS cycles to 0-1%), but measured 7% slower in
// double (12.2 against 11.3 us per launch at 3D N=32) with the larger
// scratch, so it is not used.
template <int D, int N> constexpr int col_pad() { return pad_scratch<N>(); }
template <int D, int N> constexpr int col_slots() { return scratch_slots<N>(); }

// 3D slab pass: padding of its row transforms' scratch (one spare slot
// every 8 elements) and the row pitch of its LDS planes (prec 0 double, 1
// float).  Chosen by counting each row phase's LDS bank accesses with 32
// four-byte banks serving 128 bytes per cycle (the model that reproduces
// the measured bank-conflict shares): the rows a wavefront transforms
// together must start on different banks, and a lane's padded run must
// not collide with its neighbours'.  With these, every row phase is
// conflict-free except the first stage at N = 32 (1.25 cycles per ideal
// one, against 2 for the scratch size as pitch).
template <int N> constexpr int slab_row_pad() { return N == 32 ? 8 : pad_scratch<N>(); }
template <int N> constexpr int plane_pitch(int prec) {
    return N == 32 ? 36 : (N == 64 && prec == 1 ? 72 : scratch_slots<N>());
}
// LDS slots a row transform needs: padded, the last element at N-1 + (N-1)/8.
template <int N> constexpr int slab_row_slots() { return slab_row_pad<N>() ? N + (N - 1) / slab_row_pad<N>() : N; }

// Dynamic LDS of the field-parallel column pass: 160 KB per workgroup less
// room for its static arrays.
constexpr unsigned FP_LDS_LIMIT = 140 * 1024;

// Largest workgroup of the field-parallel column pass: 1024 lanes, except
// in double where a lane needs more than the 128 registers it gets at that
// size (the compiler's resource report shows the spills): N = 128 and the
// radix-3 sizes 48 and 96, the real form (two fields per transform), and
// the fused form, whose interpolation keeps a batch of spectrum values in
// registers across the first barrier (and runs on 512 lanes anyway).
constexpr int fp_max_threads(int prec, int N, bool fused = false, bool real = false) {
    return prec == 0 && (N >= 128 || N % 3 == 0 || real) ? 512 : 1024;
}
// Row pitches (in elements) of the fused form's LDS arrays: the slab-field
// columns and staged phase rows (read by field blocks of TPT lanes, one row
// each) and the interpolation partial sums (in double written by
// matrix-core tiles, 16 lanes of a 128-byte bank cycle holding 8 slab
// fields' values of one row: with rows N + 1 elements apart they fall on
// different banks; float, whose vector form writes consecutive rows, keeps
// N + 8).
constexpr int fused_hpitch(int N) { return N + 8; }
constexpr int fused_ppitch(int prec, int N) { return N + (prec == 0 ? 1 : 8); }
// Columns per field block: 1 in 2D, else 4.
constexpr int fp_block(int d) { return d == 2 ? 1 : 4; }


constexpr int pow2_floor(int v) { int p = 1; while (2 * p <= v) p *= 2; return p; }

// Matrix-core form of the fused interpolation: the sum over x1 for one
// column is a real GEMM with rows j0 (tiles of 16), columns (slab field,
// real or imaginary part) (tiles of 16: 8 slab fields) and depth (x1, real
// or imaginary part), on 16 x 16 x 4 MFMA tiles.  With nt threads (nt / 64
// wavefronts) and ns slab fields, each tile's depth is split in the largest
// power of two of parts that still gives every part a wavefront and divides
// the N / 4 groups of four x1 values.
constexpr int mfma_tiles(int N, int ns) { return (N / 16) * ((2 * ns + 15) / 16); }
constexpr int mfma_ksplit(int N, int ns, int nt) {
    int ks = 1;
    while (2 * ks * mfma_tiles(N, ns) <= nt / 64 && (N / 4) % (2 * ks) == 0) ks *= 2;
    return ks;
}

template <int D, int N> struct Geo {
    static constexpr int TPT = FftShape<N>::TPT;
    // column pass: GB columns x IGS item slots per workgroup.  Enough slots
    // to hold every item of the common quadratures (N_r N_s = 16) in one
    // workgroup, so the sum needs no cross-workgroup step.  2D columns are
    // contiguous (one column per workgroup); 3D groups several neighbouring
    // columns per workgroup so each load row is a whole cache line.
    static constexpr int GB = D == 2 ? 1 : 8;
    static constexpr int IGS32 = D == 2 ? 16 : ((GB * TPT * 16 <= 512) ? 16 : ((GB * TPT * 8 <= 512) ? 8 : 4));
    static constexpr int IGS64 = D == 2 ? 16 : ((TPT < 12 && GB * TPT * 16 <= 512) ? 16 : ((GB * TPT * 8 <= 512) ? 8 : 4));
    // 2D slab pass: JB rows x SB fields per workgroup (JB rows of one field
    // fill a 128-byte line of the transposed output).  Small workgroups of
    // about 128 lanes spread the work over every compute unit; the forward
    // row transforms a workgroup repeats for its own fields are cheap.
    static constexpr int JB64 = N < 8 ? N : 8;
    static constexpr int JB32 = N < 16 ? N : 16;
    static constexpr int SB64 = (128 + JB64 * TPT - 1) / (JB64 * TPT);
    static constexpr int SB32 = (128 + JB32 * TPT - 1) / (JB32 * TPT);
    static constexpr int GA3 = (N < pow2_floor(256 / TPT)) ? N : pow2_floor(256 / TPT);
    // concurrent shifted fields per 3D slab-pass workgroup (LDS: SC planes,
    // the first of which also holds the slab while it is transformed)
    static constexpr int PL32 = N * plane_pitch<N>(1), PL64 = N * plane_pitch<N>(0);   // elements of one LDS plane
    static constexpr int SC32 = PL32 * 8 * 4 <= 65536 ? 4 : (PL32 * 8 * 2 <= 120000 ? 2 : 1);
    static constexpr int SC64 = PL64 * 16 * 4 <= 65536 ? 4 : (PL64 * 16 * 2 <= 65536 ? 2 : 1);
    // a second workgroup width the autotuner may take (0: none): for double
    // N = 32 a wider one (three fields per workgroup), which the plan also
    // takes when it brings the slab pass within one workgroup per compute
    // unit
    static constexpr int SC64_ALT = D == 3 && N == 32 ? 3 : 0;
    static constexpr int GF = D == 2 ? 8 : pow2_floor(256 / TPT);   // column forward
    // 3D slab pass in register form (a lane holds a whole row) for N <= 32:
    // wavefronts per workgroup
    static constexpr bool REG3_32 = D == 3 && N <= 32, REG3_64 = D == 3 && N <= 16;
    static constexpr int NWR32 = 2, NWR64 = 4;
    // slab fields per 3D slab-pass task: exactly the fields a workgroup has
    // in flight, so each task is one round (the shared slab fields are few,
    // and small tasks spread them over the chip)
    static constexpr int SPT3_64 = REG3_64 ? (64 / N) * NWR64 : SC64;
    static constexpr int SPT3_32 = REG3_32 ? (64 / N) * NWR32 : SC32;
};
}  // namespace wke
