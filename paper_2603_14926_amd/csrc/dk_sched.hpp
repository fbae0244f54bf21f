// dk_sched.hpp -- host-side builder of the lane-packed Durand-Kerner schedule.
//
// One Jacobi sweep (Section 4.2, the DK update) of a degree-n polynomial costs
// every root about n complex Horner steps plus n factors of the
// root-difference product, and all of a polynomial's roots must finish sweep
// t before any of them starts sweep t + 1.  A job is a set of whole
// polynomials swept by one W-wave workgroup (a barrier per sweep).  Inside a
// job the roots are laid out lane by lane over 64-lane items, largest degree
// first, so roots of different polynomials share a wave instead of leaving
// lanes idle; an item's loops run to the largest degree among its lanes.
// Items go to the job's waves longest first, each to the least-loaded wave.
//
// Job building, over the polynomials not yet placed:
//   * start from the largest; keep adding the next largest while the job's
//     heaviest wave stays within the cap;
//   * fill: put whole smaller polynomials into the idle lanes of the last
//     item (free: the item's length does not change), then add, as new
//     items, the largest polynomial that still fits without making the
//     heaviest wave heavier, as long as one does;
//   * the cap is L = lscale * (the largest single polynomial's heaviest wave),
//     lowered towards the end of the batch to (remaining work) / (slots W),
//     so the last jobs are short and the persistent grid drains evenly.
// Dynamic schedules order the jobs heaviest first; the kernel's workgroups
// take them from a shared counter.  Static schedules assign every job to one
// of `slots` workgroups (heaviest job first to the least-loaded workgroup,
// then moves and swaps of jobs that lower the most-loaded workgroup's total
// while any does) and store each workgroup's jobs contiguously, heaviest
// first.  Deterministic: ties go to the lower polynomial, job, wave or
// workgroup index.
#pragma once

#include <algorithm>
#include <cstdint>
#include <map>
#include <vector>

namespace mpx {

struct LaneSchedHost {
    std::vector<int> wave_off;   // njobs * W + 1
    std::vector<int> item_len;   // per item
    std::vector<int> lanes;      // per item: 64 (polynomial, root) pairs, polynomial -1 = idle
    std::vector<int> poly_off;   // njobs + 1
    std::vector<int> polys;
    std::vector<long long> job_cost;  // heaviest wave of each job (sum of item lengths)
    std::vector<int> wg_off;     // static schedules: slots + 1 job offsets per workgroup; else empty
    int njobs = 0;
};

namespace dks {

// Heaviest wave when the items of `len` (non-increasing) go, in order, to the
// least-loaded of W waves; `wave` receives the assignment when non-null.
inline long long lpt(const std::vector<int>& len, int W, std::vector<int>* wave = nullptr) {
    std::vector<long long> ld(W, 0);
    if (wave) wave->assign(len.size(), 0);
    for (size_t i = 0; i < len.size(); ++i) {
        int w = 0;
        for (int v = 1; v < W; ++v)
            if (ld[v] < ld[w]) w = v;
        ld[w] += len[i];
        if (wave) (*wave)[i] = w;
    }
    return *std::max_element(ld.begin(), ld.end());
}

// Wave loads under the same assignment.
inline std::vector<long long> lpt_loads(const std::vector<int>& len, int W) {
    std::vector<long long> ld(W, 0);
    for (size_t i = 0; i < len.size(); ++i) {
        int w = 0;
        for (int v = 1; v < W; ++v)
            if (ld[v] < ld[w]) w = v;
        ld[w] += len[i];
    }
    return ld;
}

struct Job {
    std::vector<int> lane_b, lane_r;  // layout, lane by lane (b = -1: idle lane)
    std::vector<int> polys;
    int item_len(size_t k, const std::vector<int>& deg) const { return deg[lane_b[64 * k]]; }
    size_t items() const { return (lane_b.size() + 63) / 64; }
    int spare() const { return (int)((64 - lane_b.size() % 64) % 64); }
    std::vector<int> lens(const std::vector<int>& deg) const {
        std::vector<int> l(items());
        for (size_t k = 0; k < l.size(); ++k) l[k] = item_len(k, deg);
        return l;
    }
    // Roots of b may share the last item only if b is no longer than it;
    // otherwise they start a new item (the last one's idle lanes stay idle).
    bool shares_last(int b, const std::vector<int>& deg) const {
        return spare() > 0 && deg[b] <= item_len(items() - 1, deg);
    }
    void add(int b, const std::vector<int>& deg) {
        if (spare() > 0 && !shares_last(b, deg)) {
            const int pad = spare();
            lane_b.insert(lane_b.end(), pad, -1);
            lane_r.insert(lane_r.end(), pad, 0);
        }
        polys.push_back(b);
        for (int r = 0; r < deg[b]; ++r) {
            lane_b.push_back(b);
            lane_r.push_back(r);
        }
    }
    // heaviest wave over W waves if polynomial b were added
    long long trial(int b, const std::vector<int>& deg, int W) const {
        std::vector<int> l = lens(deg);
        const long long start = shares_last(b, deg) ? (long long)lane_b.size() : 64LL * (long long)items();
        const long long used = start + deg[b];
        const size_t items2 = (size_t)((used + 63) / 64);
        while (l.size() < items2) l.push_back(deg[b]);
        return lpt(l, W);
    }
};

// Unplaced polynomials by degree; within a degree the lowest index first.
struct Pool {
    std::map<int, std::vector<int>> by;  // degree -> indices, descending (back() = lowest)
    long long count = 0;
    void put(int deg, int b) { by[deg].push_back(b); ++count; }
    void seal() {
        for (auto& kv : by) std::sort(kv.second.rbegin(), kv.second.rend());
    }
    bool empty() const { return count == 0; }
    int peek_largest() const { return by.rbegin()->second.back(); }
    int peek_smallest() const { return by.begin()->second.back(); }
    // the largest degree <= cap, or -1
    int peek_le(int cap) const {
        auto it = by.upper_bound(cap);
        if (it == by.begin()) return -1;
        --it;
        return it->second.back();
    }
    void take(int deg, int b) {
        auto it = by.find(deg);
        it->second.pop_back();
        if (it->second.empty()) by.erase(it);
        --count;
    }
};

// The largest unplaced polynomial whose addition keeps J's heaviest wave
// within lim (lowest index among equal degrees), or -1.  A polynomial that
// does not share the last item adds ceil(d / 64) items of length d, which
// the assignment puts, one after another, on the lightest wave: that is
// replayed on the current wave loads instead of a full trial.
inline int best_fit(const Job& J, const Pool& pool, long long lim, const std::vector<int>& deg,
                    int W) {
    const std::vector<long long> ld0 = lpt_loads(J.lens(deg), W);
    const long long room = lim - *std::min_element(ld0.begin(), ld0.end());
    std::vector<long long> ld;
    for (auto it = pool.by.rbegin(); it != pool.by.rend(); ++it) {
        const int d = it->first;
        if (d > lim) continue;
        const int c = it->second.back();
        if (J.shares_last(c, deg)) {
            if (J.trial(c, deg, W) <= lim) return c;
            continue;
        }
        if (d > room) continue;
        ld = ld0;
        bool fits = true;
        for (int k = 0; k < (d + 63) / 64 && fits; ++k) {
            int w = 0;
            for (int v = 1; v < W; ++v)
                if (ld[v] < ld[w]) w = v;
            ld[w] += d;
            fits = ld[w] <= lim;
        }
        if (fits) return c;
    }
    return -1;
}

// Static assignment of jobs (costs, heaviest first) to `bins` workgroups:
// each job to the least-loaded bin, then, while it lowers the most-loaded
// bin's total, the best single move of one of its jobs to another bin or
// swap with a lighter job there.  Returns each job's bin.
inline std::vector<int> assign_bins(const std::vector<long long>& cost, int bins) {
    std::vector<int> bin_of(cost.size(), 0);
    std::vector<std::vector<int>> in(bins);
    std::vector<long long> load(bins, 0);
    for (size_t j = 0; j < cost.size(); ++j) {
        int b = 0;
        for (int v = 1; v < bins; ++v)
            if (load[v] < load[b]) b = v;
        in[b].push_back((int)j);
        load[b] += cost[j];
        bin_of[j] = b;
    }
    for (size_t guard = 0; guard < 64 * cost.size() + 64; ++guard) {
        int M = 0;
        for (int v = 1; v < bins; ++v)
            if (load[v] > load[M]) M = v;
        long long best = load[M];
        int tb = -1, ta = -1, tj = -1;
        for (int b = 0; b < bins; ++b) {
            if (b == M || load[b] >= load[M]) continue;
            for (int ia = 0; ia < (int)in[M].size(); ++ia) {
                const long long ca = cost[in[M][ia]];
                const long long mv = std::max(load[M] - ca, load[b] + ca);
                if (mv < best) { best = mv; tb = b; ta = ia; tj = -1; }
                for (int ib = 0; ib < (int)in[b].size(); ++ib) {
                    const long long d = ca - cost[in[b][ib]];
                    if (d <= 0) continue;
                    const long long sw = std::max(load[M] - d, load[b] + d);
                    if (sw < best) { best = sw; tb = b; ta = ia; tj = ib; }
                }
            }
        }
        if (tb < 0) break;
        const int a = in[M][ta];
        if (tj < 0) {
            in[M].erase(in[M].begin() + ta);
            in[tb].push_back(a);
            load[M] -= cost[a];
            load[tb] += cost[a];
            bin_of[a] = tb;
        } else {
            const int c = in[tb][tj];
            in[M][ta] = c;
            in[tb][tj] = a;
            load[M] += cost[c] - cost[a];
            load[tb] += cost[a] - cost[c];
            bin_of[a] = tb;
            bin_of[c] = M;
        }
    }
    return bin_of;
}

}  // namespace dks

// deg: degrees (>= 1); W: waves per job; lscale: cap scale; slots: jobs
// resident at once on the device (for the tail cap; the number of
// workgroups of a static schedule); static_bins: build a static schedule.
// Returns false when an index would overflow the int tables.
inline bool build_lane_sched(const std::vector<int>& deg, int W, double lscale, long long slots,
                             LaneSchedHost& out, bool static_bins = false) {
    using namespace dks;
    const int N = (int)deg.size();
    Pool pool;
    long long L1 = 0, remaining = 0;
    for (int b = 0; b < N; ++b) {
        pool.put(deg[b], b);
        const long long items = (deg[b] + 63) / 64;
        L1 = std::max(L1, (items + W - 1) / W * deg[b]);
        remaining += (long long)deg[b] * deg[b];  // lane-steps; / (64 W) per wave
    }
    pool.seal();
    const long long Lmax = std::max<long long>(1, (long long)(lscale * (double)L1));
    if (slots < 1) slots = 1;
    std::vector<Job> jobs;
    std::vector<long long> cost;
    while (!pool.empty()) {
        Job J;
        int b = pool.peek_largest();
        pool.take(deg[b], b);
        J.add(b, deg);
        remaining -= (long long)deg[b] * deg[b];
        // cap: Lmax, lowered near the end of the batch (never below this
        // polynomial's own heaviest wave)
        const long long own = lpt(J.lens(deg), W);
        const long long tail = remaining / (64LL * W) / slots;
        const long long cap = std::max(own, std::min(Lmax, tail));
        while (!pool.empty()) {
            const int c = pool.peek_largest();
            if (J.trial(c, deg, W) > cap) break;
            pool.take(deg[c], c);
            J.add(c, deg);
            remaining -= (long long)deg[c] * deg[c];
        }
        // fill idle lanes of the last item, then add small polynomials as
        // new items while the heaviest wave does not grow
        long long H = lpt(J.lens(deg), W);
        for (;;) {
            if (pool.empty()) break;
            // a filler fits the idle lanes and is no longer than the last item
            const int sp = J.spare() > 0 ? std::min(J.spare(), J.item_len(J.items() - 1, deg)) : 0;
            const int c = sp > 0 ? pool.peek_le(sp) : -1;
            if (c >= 0) {
                pool.take(deg[c], c);
                J.add(c, deg);
                remaining -= (long long)deg[c] * deg[c];
                continue;
            }
            const int s = best_fit(J, pool, H, deg, W);
            if (s < 0) break;
            pool.take(deg[s], s);
            J.add(s, deg);
            remaining -= (long long)deg[s] * deg[s];
            H = lpt(J.lens(deg), W);
        }
        cost.push_back(H);
        jobs.push_back(std::move(J));
    }
    // heaviest first (stable: build order on ties)
    std::vector<int> ord(jobs.size());
    for (size_t j = 0; j < ord.size(); ++j) ord[j] = (int)j;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return cost[a] > cost[c]; });
    std::vector<int> wg_off;
    if (static_bins) {
        if (slots > INT32_MAX / 2) return false;
        const int bins = (int)slots;
        std::vector<long long> sorted_cost(ord.size());
        for (size_t j = 0; j < ord.size(); ++j) sorted_cost[j] = cost[ord[j]];
        const std::vector<int> bin_of = assign_bins(sorted_cost, bins);
        // group by workgroup, keeping heaviest first inside each
        std::vector<int> pos(ord.size());
        for (size_t j = 0; j < pos.size(); ++j) pos[j] = (int)j;
        std::stable_sort(pos.begin(), pos.end(), [&](int a, int c) {
            return bin_of[a] != bin_of[c] ? bin_of[a] < bin_of[c] : sorted_cost[a] > sorted_cost[c];
        });
        std::vector<int> grouped(ord.size());
        for (size_t j = 0; j < pos.size(); ++j) grouped[j] = ord[pos[j]];
        wg_off.assign(bins + 1, 0);
        for (size_t j = 0; j < pos.size(); ++j) ++wg_off[bin_of[pos[j]] + 1];
        for (int b = 0; b < bins; ++b) wg_off[b + 1] += wg_off[b];
        ord.swap(grouped);
    }
    out = LaneSchedHost{};
    out.wg_off = wg_off;
    out.njobs = (int)jobs.size();
    out.wave_off.push_back(0);
    out.poly_off.push_back(0);
    long long total_items = 0;
    for (const Job& J : jobs) total_items += (long long)J.items();
    if (total_items * 64 * 2 > (long long)INT32_MAX || (long long)jobs.size() * W + 1 > INT32_MAX)
        return false;
    for (int j : ord) {
        const Job& J = jobs[j];
        const std::vector<int> len = J.lens(deg);
        std::vector<int> wave;
        lpt(len, W, &wave);
        for (int w = 0; w < W; ++w) {
            for (size_t k = 0; k < len.size(); ++k) {
                if (wave[k] != w) continue;
                out.item_len.push_back(len[k]);
                for (int l = 0; l < 64; ++l) {
                    const size_t p = 64 * k + l;
                    out.lanes.push_back(p < J.lane_b.size() ? J.lane_b[p] : -1);
                    out.lanes.push_back(p < J.lane_b.size() ? J.lane_r[p] : 0);
                }
            }
            out.wave_off.push_back((int)out.item_len.size());
        }
        out.polys.insert(out.polys.end(), J.polys.begin(), J.polys.end());
        out.poly_off.push_back((int)out.polys.size());
        out.job_cost.push_back(cost[j]);
    }
    return true;
}

}  // namespace mpx
