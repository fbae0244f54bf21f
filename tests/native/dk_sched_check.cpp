// CPU check of the lane-packed Durand-Kerner schedule builder (host code of
// the library, compiled here with g++): every root of every polynomial is on
// exactly one lane of one item of the job that lists its polynomial, no lane
// holds a polynomial longer than its item, items of a job are split into W
// waves, and the recorded job cost is the heaviest wave.
#include "../../paper_2603_14926_amd/csrc/dk_sched.hpp"

#include <vector>

extern "C" int dk_sched_check(const int* degs, int n, int W, double lscale, long long slots,
                              double* stats) {
    std::vector<int> deg(degs, degs + n);
    mpx::LaneSchedHost S;
    if (!mpx::build_lane_sched(deg, W, lscale, slots, S)) return -1;
    if ((int)S.wave_off.size() != S.njobs * W + 1 || (int)S.poly_off.size() != S.njobs + 1) return -2;
    if (S.lanes.size() != S.item_len.size() * 128 || S.polys.size() != (size_t)n) return -3;
    std::vector<int> job_of(n, -1);
    for (int j = 0; j < S.njobs; ++j)
        for (int q = S.poly_off[j]; q < S.poly_off[j + 1]; ++q) {
            const int b = S.polys[q];
            if (b < 0 || b >= n || job_of[b] != -1) return -4;   // each polynomial in one job
            job_of[b] = j;
        }
    std::vector<std::vector<char>> seen(n);
    for (int b = 0; b < n; ++b) seen[b].assign(deg[b], 0);
    double useful = 0, issued = 0;
    for (int b = 0; b < n; ++b) useful += (double)deg[b] * deg[b];
    for (int j = 0; j < S.njobs; ++j) {
        long long heaviest = 0;
        for (int w = 0; w < W; ++w) {
            long long load = 0;
            for (int i = S.wave_off[j * W + w]; i < S.wave_off[j * W + w + 1]; ++i) {
                load += S.item_len[i];
                issued += 64.0 * S.item_len[i];
                for (int l = 0; l < 64; ++l) {
                    const int b = S.lanes[128LL * i + 2 * l], r = S.lanes[128LL * i + 2 * l + 1];
                    if (b < 0) continue;
                    if (b >= n || job_of[b] != j || r < 0 || r >= deg[b]) return -5;
                    if (deg[b] > S.item_len[i] || seen[b][r]) return -6;
                    seen[b][r] = 1;
                }
            }
            if (load > heaviest) heaviest = load;
        }
        if (heaviest != S.job_cost[j]) return -7;
        if (j > 0 && S.job_cost[j] > S.job_cost[j - 1]) return -8;       // heaviest first
    }
    for (int b = 0; b < n; ++b)
        for (char c : seen[b])
            if (!c) return -9;
    stats[0] = S.njobs;
    stats[1] = useful / issued;      // share of issued lane-steps that are a root's own steps
    return 0;
}
