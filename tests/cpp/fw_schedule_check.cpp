// Host-logic check of the blocked Floyd-Warshall schedule (fw_schedule.h),
// at the level of 64x64 blocks: every block (I,J) must receive the update of
// every pivot block K exactly once and in increasing K, each update reading
// its operands (I,K) and (K,J) in the state the sequential blocked order
// reads them in (every pivot block up to K applied, none after), and no
// launch may write a block that the same launch reads.
#include <cstdio>
#include <set>
#include <utility>
#include <vector>

#include "fw_schedule.h"

namespace {

int fails = 0;

void fail(const char* what, int nb, bool quads, int step, int I, int J, int K) {
    if (fails < 20)
        std::printf("nb=%d quads=%d step %d: %s at block (%d,%d) pivot %d\n", nb, (int)quads, step, what, I,
                    J, K);
    ++fails;
}

struct Model {
    int nb;
    std::vector<int> done;  // pivot blocks applied to (I,J): always 0..done-1
    explicit Model(int nb_) : nb(nb_), done((size_t)nb_ * nb_, 0) {}
    int& at(int I, int J) { return done[(size_t)I * nb + J]; }
};

// Targets of a phase-3 style update with the pivot blocks Ks (in order).
void apply(Model& M, const std::vector<std::pair<int, int>>& targets, const std::vector<int>& Ks, bool quads,
           int step) {
    const int nb = M.nb;
    std::set<std::pair<int, int>> seen, reads;
    for (auto [I, J] : targets) {
        if (I < 0 || J < 0 || I >= nb || J >= nb) { fail("target out of range", nb, quads, step, I, J, Ks[0]); continue; }
        if (!seen.insert({I, J}).second) fail("target twice in one launch", nb, quads, step, I, J, Ks[0]);
        for (int K : Ks) {
            reads.insert({I, K});
            reads.insert({K, J});
        }
    }
    for (auto t : seen)
        if (reads.count(t)) fail("launch reads a block it writes", nb, quads, step, t.first, t.second, Ks[0]);
    // operands as the sequential order reads them, all at the launch's start
    for (auto [I, J] : seen)
        for (int K : Ks) {
            if (I == K || J == K) { fail("phase-3 update of the pivot's own row/column", nb, quads, step, I, J, K); continue; }
            if (M.at(I, K) != K + 1) fail("operand (I,K) in the wrong state", nb, quads, step, I, J, K);
            if (M.at(K, J) != K + 1) fail("operand (K,J) in the wrong state", nb, quads, step, I, J, K);
        }
    for (auto [I, J] : seen)
        for (int K : Ks) {
            if (M.at(I, J) != K) fail("pivot applied out of order", nb, quads, step, I, J, K);
            M.at(I, J) = K + 1;
        }
}

void check(int nb, bool quads) {
    Model M(nb);
    const auto steps = btas::fw_schedule(nb, quads);
    for (size_t si = 0; si < steps.size(); ++si) {
        const btas::FwStep& st = steps[si];
        const int step = (int)si;
        std::vector<std::pair<int, int>> tg;
        switch (st.kind) {
            case btas::FW_PHASE12: {
                const int K = st.kb;
                // phase 1: the diagonal block; phase 2: its row and column
                // against the finished diagonal block
                if (M.at(K, K) != K) fail("phase 1 out of order", nb, quads, step, K, K, K);
                M.at(K, K) = K + 1;
                for (int X = 0; X < nb; ++X) {
                    if (X == K) continue;
                    if (M.at(K, X) != K) fail("phase 2 (row) out of order", nb, quads, step, K, X, K);
                    if (M.at(X, K) != K) fail("phase 2 (column) out of order", nb, quads, step, X, K, K);
                    M.at(K, X) = K + 1;
                    M.at(X, K) = K + 1;
                }
                break;
            }
            case btas::FW_UPDATE: {
                const unsigned cnt = btas::update_blocks(st.u);
                for (unsigned t = 0; t < cnt; ++t) {
                    int I, J;
                    btas::select_block(st.u, (int)t, I, J);
                    tg.push_back({I, J});
                }
                apply(M, tg, {st.u.kb}, quads, step);
                break;
            }
            case btas::FW_BAND: {
                const long cnt = btas::band_blocks(st.b);
                for (long t = 0; t < cnt; ++t) {
                    int I, J;
                    btas::select_band(st.b, (int)t, I, J);
                    tg.push_back({I, J});
                }
                apply(M, tg, {st.b.kb}, quads, step);
                break;
            }
            case btas::FW_PAIR:
            case btas::FW_QUAD: {
                const bool quad = st.kind == btas::FW_QUAD;
                const int nt = (nb + 1) / 2;  // 128x128 tiles per dimension
                const long tiles = quad ? (long)(nt - 2) * (nt - 2) : (long)(nt - 1) * (nt - 1);
                for (long t = 0; t < tiles; ++t) {
                    int m0, n0;
                    if (quad) btas::quad_tile((int)t, st.q, nt, m0, n0);
                    else btas::pair_tile((int)t, st.q, nt, m0, n0);
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b) {
                            const int I = m0 / btas::FW_B + a, J = n0 / btas::FW_B + b;
                            if (I < nb && J < nb) tg.push_back({I, J});
                        }
                }
                std::vector<int> Ks;
                for (int j = 0; j < (quad ? 4 : 2); ++j)
                    if (st.kb + j < nb) Ks.push_back(st.kb + j);
                apply(M, tg, Ks, quads, step);
                break;
            }
        }
    }
    for (int I = 0; I < nb; ++I)
        for (int J = 0; J < nb; ++J)
            if (M.at(I, J) != nb) fail("block not fully relaxed at the end", nb, quads, -1, I, J, M.at(I, J));
}

}  // namespace

int main() {
    int schedules = 0;
    for (int nb = 1; nb <= 40; ++nb) {
        check(nb, false);
        ++schedules;
        if (nb % 2 == 0) {  // groups of four need every 128x128 tile full
            check(nb, true);
            ++schedules;
        }
    }
    check(256, true);  // n = 16384
    check(256, false);
    std::printf("schedules checked: %d\n", schedules + 2);
    std::printf("fw schedule failures: %d\n", fails);
    return fails != 0;
}
