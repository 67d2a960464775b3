// Host-side check of the LDS layout arithmetic the streamed kernels rely on
// (built and run by test_lds_layouts.py).  For every exchange of the fused
// row and column transforms of 256..2048 points, the natural-order exchange
// of the mirror-paired column tiles and the full transforms of their
// emission round trip, it checks that
//   - the base-plus-offset forms (lpos_step, lpos_run, lpos_write) equal the
//     position of the full index, for every element a pass touches;
//   - each padded layout maps the L elements to distinct positions below
//     pad_len(L, A);
//   - the pad pad_of picks keeps the writing pass free of bank conflicts
//     within 32 lanes, and each padded layout uses at most the pad the tile
//     sizes (PairLayout::AMAX) allow for.
#include <cstdio>

#include "mf_streamed_fft.hpp"

using namespace mf;

static int fails = 0, checks = 0;
#define CHECK(c, ...)                    \
    do {                                 \
        ++checks;                        \
        if (!(c)) {                      \
            if (++fails <= 20) {         \
                std::printf(__VA_ARGS__); \
                std::printf("\n");       \
            }                            \
        }                                \
    } while (0)

template <int L, int A>
void check_layout() {
    if constexpr (A >= 0) {
        static bool seen[2 * 4096];
        for (auto& b : seen) b = false;
        for (int i = 0; i < L; ++i) {
            const unsigned p = lpos<A>((unsigned)i);
            CHECK((int)p < pad_len(L, A), "L=%d A=%d: element %d at %u past pad_len %d", L, A, i, p, pad_len(L, A));
            CHECK(!seen[p], "L=%d A=%d: position %u taken twice", L, A, p);
            seen[p] = true;
        }
    }
}

// One pass: reads j + r NT in layout AI, writes o + r NS in layout AO.
template <int L, int R, int NS, int AI, int AO>
void check_pass() {
    constexpr int NT = L / R;
    for (int j = 0; j < NT; ++j)
        for (int r = 0; r < R; ++r) {
            CHECK((lpos_step<AI, NT>(j, r)) == lpos<AI>(j + r * NT), "read L=%d R=%d NS=%d A=%d j=%d r=%d", L, R, NS,
                  AI, j, r);
            const unsigned o = (j / NS) * NS * R + j % NS;
            CHECK((lpos_write<AO, R, NS>(o, r)) == lpos<AO>(o + r * NS), "write L=%d R=%d NS=%d A=%d j=%d r=%d", L, R,
                  NS, AO, j, r);
        }
    if constexpr (AO >= 0) CHECK(pad_writes_ok(L, R, NS, AO), "L=%d R=%d NS=%d: pad %d has write conflicts", L, R, NS, AO);
    check_layout<L, AO>();
}

// The middle passes of passes_before<L, RM, NS, TAIL, ..., AI>.
template <int L, int RM, int NS, int TAIL, int AI>
void check_chain() {
    if constexpr (NS * RM * TAIL <= L && NS * TAIL < L) {
        constexpr int AO = AI >= 0 ? pad_of(L, RM, NS) : -1;
        check_pass<L, RM, NS, AI, AO>();
        check_chain<L, RM, NS * RM, TAIL, AO>();
    }
}

// The passes of stockham_fft<L, NS, ..., AI, AOUT>.
template <int L, int NS, int AI, int AOUT>
void check_fft() {
    if constexpr (NS < L) {
        constexpr int R = next_radix<L / NS>();
        constexpr int AO = NS * R == L ? AOUT : (AI >= 0 ? pad_of(L, R, NS) : -1);
        CHECK((AO <= PairLayout<L, 8>::AMAX), "L=%d NS=%d: emission pad %d beyond the tile's", L, NS, AO);
        check_pass<L, R, NS, AI, AO>();
        check_fft<L, NS * R, AO, AOUT>();
    }
}

template <int L>
void check_length() {
    constexpr int RL = last_radix<L>(), RM = middle_radix<L>();
    constexpr int A1 = pad_of(L, 16, 1), AC = pad_after(L, RM, 16, RL, A1);
    constexpr int AF = pad_of(L, RL, 1), AD = pad_after(L, RM, RL, 16, AF);
    constexpr int AN = pad_of(L, RL, L / RL);
    // the first pass of each direction (stage A / phase A, stage C's write)
    for (int j = 0; j < L / 16; ++j)
        for (int r = 0; r < 16; ++r) CHECK((lpos_run<A1, 16>(j, r)) == lpos<A1>(16 * j + r), "run16 L=%d", L);
    for (int j = 0; j < L / RL; ++j)
        for (int r = 0; r < RL; ++r) CHECK((lpos_run<AF, RL>(j, r)) == lpos<AF>(RL * j + r), "runRL L=%d", L);
    CHECK(pad_writes_ok(L, 16, 1, A1), "L=%d: first forward pass conflicts", L);
    CHECK(pad_writes_ok(L, RL, 1, AF), "L=%d: first inverse pass conflicts", L);
    check_layout<L, A1>();
    check_layout<L, AF>();
    // middle passes of both directions
    check_chain<L, RM, 16, RL, A1>();
    check_chain<L, RM, RL, 16, AF>();
    // the fused kernels' register stages read AC (j + r L/RL) and AD (j + r L/16)
    for (int j = 0; j < L / RL; ++j)
        for (int r = 0; r < RL; ++r) CHECK((lpos_step<AC, L / RL>(j, r)) == lpos<AC>(j + r * (L / RL)), "AC L=%d", L);
    for (int j = 0; j < L / 16; ++j)
        for (int r = 0; r < 16; ++r) CHECK((lpos_step<AD, L / 16>(j, r)) == lpos<AD>(j + r * (L / 16)), "AD L=%d", L);
    // mirror-paired tiles: the last forward pass leaves natural order in AN,
    // the first inverse pass reads it; the emission round trip runs whole
    // transforms from AN to AN
    check_pass<L, RL, L / RL, AC, AN>();
    check_pass<L, RL, 1, AN, AF>();
    check_fft<L, 1, AN, AN>();
    // every pad the transforms use fits the tiles' rows
    constexpr int AMAX = PairLayout<L, 8>::AMAX;
    CHECK(A1 <= AMAX && AC <= AMAX && AF <= AMAX && AD <= AMAX && AN <= AMAX, "L=%d: pad beyond AMAX %d", L, AMAX);
    std::printf("L=%4d  A1=%d AC=%d AN=%d AF=%d AD=%d  tile stride (TC=4/8/16): %d/%d/%d, conflicts %d/%d/%d\n", L, A1,
                AC, AN, AF, AD, PairLayout<L, 4>::SEG, PairLayout<L, 8>::SEG, PairLayout<L, 16>::SEG,
                tile_conflicts(4, PairLayout<L, 4>::SEG, A1, AD), tile_conflicts(8, PairLayout<L, 8>::SEG, A1, AD),
                tile_conflicts(16, PairLayout<L, 16>::SEG, A1, AD));
}

int main() {
    check_length<256>();
    check_length<512>();
    check_length<1024>();
    check_length<2048>();
    std::printf("%d checks, %d failures\n", checks, fails);
    return fails == 0 ? 0 : 1;
}
