// CPU check of the lane-packed Durand-Kerner schedule builder (host code of
// the library, compiled here with g++): every root of every polynomial is on
// exactly one lane of one item of the job that lists its polynomial, no lane
// holds a polynomial longer than its item, items of a job are split into W
// waves, the recorded job cost is the heaviest wave, and jobs come heaviest
// first (static schedules: every job in exactly one workgroup's contiguous
// range, heaviest first inside it).  stats: jobs, share of issued lane-steps
// that are roots' own steps, in-job balance (sum of wave loads over W times
// the heaviest), and the makespan in lane-steps per wave (static: the most
// loaded workgroup; dynamic: jobs in order to the earliest-free workgroup)
// over the even share of all wave loads.
#include "../../paper_2603_14926_amd/csrc/dk_sched.hpp"

#include <algorithm>
#include <vector>

extern "C" int dk_sched_check(const int* degs, int n, int W, double lscale, long long slots,
                              int static_bins, double* stats) {
    std::vector<int> deg(degs, degs + n);
    mpx::LaneSchedHost S;
    if (!mpx::build_lane_sched(deg, W, lscale, slots, S, static_bins != 0)) return -1;
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
    double useful = 0, issued = 0, wave_sum = 0;
    for (int b = 0; b < n; ++b) useful += (double)deg[b] * deg[b];
    for (int j = 0; j < S.njobs; ++j) {
        long long heaviest = 0, wave_total = 0;
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
            wave_total += load;
        }
        if (heaviest != S.job_cost[j]) return -7;
        wave_sum += wave_total;
    }
    for (int b = 0; b < n; ++b)
        for (char c : seen[b])
            if (!c) return -9;
    long long makespan = 0, cost_sum = 0;
    for (long long c : S.job_cost) cost_sum += c;
    if (static_bins) {
        if ((long long)S.wg_off.size() != slots + 1 || S.wg_off[0] != 0 || S.wg_off[slots] != S.njobs)
            return -10;
        for (long long g = 0; g < slots; ++g) {
            if (S.wg_off[g + 1] < S.wg_off[g]) return -11;
            long long load = 0;
            for (int j = S.wg_off[g]; j < S.wg_off[g + 1]; ++j) {
                if (j > S.wg_off[g] && S.job_cost[j] > S.job_cost[j - 1]) return -8;
                load += S.job_cost[j];
            }
            makespan = std::max(makespan, load);
        }
    } else {
        if (!S.wg_off.empty()) return -10;
        std::vector<long long> fin(slots, 0);
        for (int j = 0; j < S.njobs; ++j) {
            if (j > 0 && S.job_cost[j] > S.job_cost[j - 1]) return -8;   // heaviest first
            auto it = std::min_element(fin.begin(), fin.end());
            *it += S.job_cost[j];
            makespan = std::max(makespan, *it);
        }
    }
    stats[0] = S.njobs;
    stats[1] = useful / issued;      // share of issued lane-steps that are a root's own steps
    stats[2] = wave_sum / ((double)W * (double)cost_sum);
    stats[3] = (double)makespan / (wave_sum / ((double)W * (double)slots));
    return 0;
}
