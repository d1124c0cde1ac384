// Blocked Floyd-Warshall: which blocks each launch covers, and the order of
// the launches (Sec. IV, Algorithm 2's relaxations grouped by pivot blocks).
//
// Host and device code share these definitions: the launches read the
// selectors, fw_schedule() lists the launches, and a host-side check walks
// the schedule block by block (every block gets every pivot block's update
// once, in pivot order, from operands in the state the sequential blocked
// order reads them in).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace btas {

constexpr int FW_B = 64;  // pivot block edge

// Which 64x64 blocks an update launch covers; every covered block (I,J) gets
// D_IJ <- D_IJ (+) D_I,kb (.) D_kb,J with the k-range of pivot block kb.
//   full:  every I != kb, J != kb                       ((nb-1)^2 blocks)
//   strip: block-row rb (J != skip) and block-column rb (I != rb, I != skip)
//          (2nb-3 blocks; rb != skip)
struct UpdateSel {
    int kb, nb;
    int rb, skip;  // rb < 0: full
};

__host__ __device__ __forceinline__ void select_block(const UpdateSel& u, int t, int& I, int& J) {
    if (u.rb < 0) {
        I = t / (u.nb - 1);
        J = t % (u.nb - 1);
        I += I >= u.kb ? 1 : 0;
        J += J >= u.kb ? 1 : 0;
    } else if (t < u.nb - 1) {
        I = u.rb;
        J = t + (t >= u.skip ? 1 : 0);
    } else {
        const int lo = u.rb < u.skip ? u.rb : u.skip, hi = u.rb < u.skip ? u.skip : u.rb;
        I = t - (u.nb - 1);
        I += I >= lo ? 1 : 0;
        I += I >= hi ? 1 : 0;
        J = u.rb;
    }
}

__host__ __device__ __forceinline__ unsigned update_blocks(const UpdateSel& u) {
    return u.rb < 0 ? (unsigned)((long)(u.nb - 1) * (u.nb - 1)) : (unsigned)(2 * u.nb - 3);
}

// Strips of a group of pivot blocks: every block (I,J) with I and J outside
// [ex_lo, ex_hi) and I or J inside [band_lo, band_hi) gets the update of
// pivot block kb (which lies in [ex_lo, ex_hi)).  The two ranges are
// adjacent, so their union is one range.
struct BandSel {
    int kb, nb;
    int band_lo, band_hi, ex_lo, ex_hi;
};

__host__ __device__ __forceinline__ long band_blocks(const BandSel& u) {
    const long bw = u.band_hi - u.band_lo, a = u.nb - (u.ex_hi - u.ex_lo);
    return a * a - (a - bw) * (a - bw);
}

// t < bw*a: the band's rows, every allowed column; then the band's columns
// for the allowed rows outside the band.
__host__ __device__ __forceinline__ void select_band(const BandSel& u, int t, int& I, int& J) {
    const int bw = u.band_hi - u.band_lo, exw = u.ex_hi - u.ex_lo, a = u.nb - exw;
    const int u_lo = u.band_lo < u.ex_lo ? u.band_lo : u.ex_lo;
    if (t < bw * a) {
        I = u.band_lo + t / a;
        const int c = t % a;
        J = c < u.ex_lo ? c : c + exw;
    } else {
        t -= bw * a;
        const int r = t / bw;
        I = r < u_lo ? r : r + bw + exw;
        J = u.band_lo + t % bw;
    }
}

// Pivot-pair update: every 128x128 tile (I,J) outside tile-row and
// tile-column sb gets D_IJ <- D_IJ (+) D_I,P (.) D_P,J, P the 128 pivots of
// blocks 2sb and 2sb+1 (fewer at a ragged end): both blocks' updates of
// the same entries in one pass.
__host__ __device__ __forceinline__ void pair_tile(int t, int sb, int nb2, int& m0, int& n0) {
    int I = t / (nb2 - 1), J = t % (nb2 - 1);
    I += I >= sb ? 1 : 0;
    J += J >= sb ? 1 : 0;
    m0 = I * 2 * FW_B;
    n0 = J * 2 * FW_B;
}

// Group update (fp32, n a multiple of 128): every 128x128 tile outside the
// 256-row band and 256-column band of group q gets
// D_IJ <- D_IJ (+) D_I,P (.) D_P,J, P the group's 256 pivots (blocks 4q..4q+3).
__host__ __device__ __forceinline__ void quad_tile(int t, int q, int nt, int& m0, int& n0) {
    int I = t / (nt - 2), J = t % (nt - 2);
    I += I >= 2 * q ? 2 : 0;
    J += J >= 2 * q ? 2 : 0;
    m0 = I * 2 * FW_B;
    n0 = J * 2 * FW_B;
}

// One launch of the blocked schedule.
enum FwStepKind {
    FW_PHASE12,  // phases 1-2 of pivot block kb (its diagonal block, then its row and column)
    FW_UPDATE,   // phase 3 of pivot block u.kb on the blocks u selects
    FW_BAND,     // phase 3 of pivot block b.kb on the blocks b selects
    FW_PAIR,     // phase 3 of pivot blocks 2q, 2q+1 on the 128x128 tiles outside their rows and columns
    FW_QUAD,     // phase 3 of pivot blocks 4q..4q+3 on the 128x128 tiles outside their rows and columns
};

struct FwStep {
    FwStepKind kind;
    int kb, q;
    UpdateSel u;
    BandSel b;
};

// The launches for nb pivot blocks.  quads: groups of four (every 128x128
// tile full, so nb is even); otherwise pairs.  Either way an odd last block
// runs the three plain phases.
//
// Pair (K0, K1): phases 1-2 of K0; K0's update of block-row and block-column
// K1; phases 1-2 of K1; one k=128 update of every tile outside rows/columns
// K0, K1 (reading row/column K0 as phase 2 of K0 left them, row/column K1 as
// phase 2 of K1 left them); then K1's update of block-row and block-column
// K0 (deferred so that the fused update read their earlier values).
//
// Group of four (K0..K3): after phases 1-2 of Kj, Kj's update of the
// block-rows and block-columns of K(j+1)..K3; one k=256 update of every tile
// outside the group's rows and columns; then, for m = 1..3 in order, Km's
// update of the block-rows and block-columns of K0..K(m-1), outside the rows
// and columns of Km..K3.
inline std::vector<FwStep> fw_schedule(int nb, bool quads) {
    std::vector<FwStep> st;
    auto phase12 = [&](int kb) { st.push_back({FW_PHASE12, kb, 0, {}, {}}); };
    auto update = [&](UpdateSel u) { st.push_back({FW_UPDATE, u.kb, 0, u, {}}); };
    auto band = [&](BandSel b) { st.push_back({FW_BAND, b.kb, 0, {}, b}); };
    int kb = 0;
    if (quads) {
        for (; kb + 4 <= nb; kb += 4) {
            for (int j = 0; j < 4; ++j) {
                phase12(kb + j);
                if (j < 3) band(BandSel{kb + j, nb, kb + j + 1, kb + 4, kb + j, kb + j + 1});
            }
            st.push_back({FW_QUAD, kb, kb / 4, {}, {}});
            for (int m = 1; m < 4; ++m) band(BandSel{kb + m, nb, kb, kb + m, kb + m, kb + 4});
        }
    }
    for (; kb + 1 < nb; kb += 2) {
        phase12(kb);
        update(UpdateSel{kb, nb, kb + 1, kb});
        phase12(kb + 1);
        st.push_back({FW_PAIR, kb, kb / 2, {}, {}});
        update(UpdateSel{kb + 1, nb, kb, kb + 1});
    }
    if (kb < nb) {
        phase12(kb);
        if (nb > 1) update(UpdateSel{kb, nb, -1, -1});
    }
    return st;
}

}  // namespace btas
