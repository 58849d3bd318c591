// Host check of the persistent batch queue: enumerates the items of random
// runs phase by phase (the definition), then compares every decoded item with
// it and checks that each dependency has a smaller item number.  Finally a
// random scheduler with W workers pulls items in order and must finish.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
#include "gsn_queue.hpp"

using namespace gsn;

int main()
{
    std::mt19937 rng(12345);
    int failures = 0;
    for (int trial = 0; trial < 300; ++trial) {
        const int count = 1 + rng() % 9;
        const long long nsteps = rng() % 5;
        std::vector<std::vector<unsigned>> tiles(Q_NKIND, std::vector<unsigned>(count));
        for (int i = 0; i < count; ++i) {
            const unsigned em = 1 + rng() % 4, lm = 1 + rng() % 5, lk = 1 + rng() % 6, ld = 1 + rng() % 3;
            tiles[Q_ENTRY][i] = em; tiles[Q_EXIT][i] = em;
            tiles[Q_KIN_HALF][i] = lm; tiles[Q_KIN_FULL][i] = lm;
            tiles[Q_DENSITY][i] = ld; tiles[Q_PHASE][i] = ld;
            tiles[Q_KERNEL][i] = lk;
        }
        std::vector<unsigned> prefix(Q_NKIND * (count + 1));
        for (int k = 0; k < Q_NKIND; ++k) {
            prefix[k * (count + 1)] = 0;
            for (int i = 0; i < count; ++i) prefix[k * (count + 1) + i + 1] = prefix[k * (count + 1) + i] + tiles[k][i];
        }
        QTables T{count, nsteps, prefix.data()};
        // the definition: phases in order, instances in order, tiles in order
        std::vector<int> phase_kinds = {Q_ENTRY, Q_KIN_HALF};
        for (long long s = 0; s < nsteps; ++s) {
            phase_kinds.push_back(Q_DENSITY); phase_kinds.push_back(Q_KERNEL); phase_kinds.push_back(Q_PHASE);
            phase_kinds.push_back(s + 1 < nsteps ? Q_KIN_FULL : Q_KIN_HALF);
        }
        phase_kinds.push_back(Q_EXIT);
        struct Ref { int kind, inst, tile; unsigned long long need; };
        std::vector<Ref> ref;
        std::vector<unsigned long long> done_before(count, 0);
        for (int k : phase_kinds) {
            std::vector<unsigned long long> snap = done_before;
            for (int i = 0; i < count; ++i)
                for (unsigned t = 0; t < tiles[k][i]; ++t) ref.push_back({k, i, (int)t, snap[i]});
            for (int i = 0; i < count; ++i) done_before[i] += tiles[k][i];
        }
        if (qtotal_items(T) != ref.size()) { ++failures; std::printf("total mismatch\n"); continue; }
        std::vector<unsigned long long> issued(count, 0);   // items of instance i numbered before x
        for (size_t x = 0; x < ref.size(); ++x) {
            const QItem it = qdecode(T, x);
            const Ref &r = ref[x];
            if (it.kind != r.kind || it.inst != r.inst || it.tile != r.tile || it.need != r.need) {
                ++failures;
                std::printf("trial %d item %zu: got (%d,%d,%d,%llu) want (%d,%d,%d,%llu)\n", trial, x, it.kind, it.inst,
                            it.tile, it.need, r.kind, r.inst, r.tile, r.need);
                break;
            }
            if (it.need > issued[it.inst]) { ++failures; std::printf("dependency not earlier\n"); break; }
            issued[it.inst] += 1;
        }
        // random in-order scheduler: W workers, each holds one item until its need is met
        const int W = 1 + rng() % 6;
        std::vector<unsigned long long> completed(count, 0);
        std::vector<long long> hold(W, -1);
        unsigned long long head = 0, finished = 0;
        long long guard = 0;
        while (finished < ref.size() && guard++ < 10000000) {
            const int w = rng() % W;
            if (hold[w] < 0) {
                if (head < ref.size()) hold[w] = (long long)head++;
                continue;
            }
            const QItem it = qdecode(T, (unsigned long long)hold[w]);
            if (completed[it.inst] >= it.need) {
                completed[it.inst] += 1;
                finished += 1;
                hold[w] = -1;
            }
        }
        if (finished != ref.size()) { ++failures; std::printf("trial %d: scheduler stuck\n", trial); }
    }
    std::printf("failures %d\n", failures);
    return failures ? 1 : 0;
}
