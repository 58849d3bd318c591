// gsn_queue.hpp -- work items of the persistent batched solver.
//
// A run of nsteps steps over `count` instances is a sequence of phases
//   q = 0: x entry FFT,  q = 1: half kinetic,
//   q = 2 + 4s + {0,1,2,3}: density, kernel, phase, kinetic (full, or half
//                           for the last step),   s = 0 .. nsteps-1,
//   q = 2 + 4 nsteps: x exit FFT.
// Items are numbered phase by phase; inside a phase instance by instance;
// inside an instance tile by tile.  Item (q, i, t) may start once instance i
// has completed every tile of every earlier phase ("need"), which the
// persistent kernel tracks with one monotone counter per instance.  Items are
// handed out in increasing order, so every item an item depends on has been
// handed to a running block first: the queue cannot deadlock.
#pragma once
#include <hip/hip_runtime.h>

namespace gsn {

// phase kinds (order inside a step matters: density, kernel, phase, kinetic)
enum QKind { Q_ENTRY = 0, Q_KIN_HALF = 1, Q_DENSITY = 2, Q_KERNEL = 3, Q_PHASE = 4, Q_KIN_FULL = 5, Q_EXIT = 6,
             Q_NKIND = 7 };

struct QTables {
    int count;          // instances
    long long nsteps;
    // per kind: exclusive prefix over instances of the tiles of that kind
    // (prefix[kind * (count + 1) + i]); total = prefix[kind * (count + 1) + count]
    const unsigned *prefix;
};

struct QItem {
    int kind, inst, tile;
    unsigned long long need;   // tiles of instance inst that must be complete first
};

__host__ __device__ inline unsigned qtotal(const QTables &T, int kind)
{
    return T.prefix[kind * (T.count + 1) + T.count];
}

__host__ __device__ inline unsigned qtiles(const QTables &T, int kind, int i)
{
    return T.prefix[kind * (T.count + 1) + i + 1] - T.prefix[kind * (T.count + 1) + i];
}

__host__ __device__ inline unsigned long long qtotal_items(const QTables &T)
{
    const unsigned long long step = (unsigned long long)qtotal(T, Q_DENSITY) + qtotal(T, Q_KERNEL) +
                                    qtotal(T, Q_PHASE) + qtotal(T, Q_KIN_FULL);
    return (unsigned long long)qtotal(T, Q_ENTRY) + qtotal(T, Q_KIN_HALF) + step * T.nsteps + qtotal(T, Q_EXIT);
}

// Decode item number x (< qtotal_items) into (kind, instance, tile, need).
__host__ __device__ inline QItem qdecode(const QTables &T, unsigned long long x)
{
    QItem it;
    const unsigned long long te = qtotal(T, Q_ENTRY), tk = qtotal(T, Q_KIN_HALF);
    const unsigned long long td = qtotal(T, Q_DENSITY), tr = qtotal(T, Q_KERNEL), tp = qtotal(T, Q_PHASE);
    const unsigned long long tf = qtotal(T, Q_KIN_FULL);
    const unsigned long long step = td + tr + tp + tf;
    long long s = -1;   // step index (-1: before the steps; nsteps: exit)
    unsigned long long off;
    int kind;
    if (x < te) {
        kind = Q_ENTRY;
        off = x;
    } else if (x < te + tk) {
        kind = Q_KIN_HALF;
        off = x - te;
    } else if (x < te + tk + step * (unsigned long long)T.nsteps) {
        const unsigned long long r0 = x - te - tk;
        s = (long long)(r0 / step);
        unsigned long long r = r0 - (unsigned long long)s * step;
        if (r < td) { kind = Q_DENSITY; off = r; }
        else if (r < td + tr) { kind = Q_KERNEL; off = r - td; }
        else if (r < td + tr + tp) { kind = Q_PHASE; off = r - td - tr; }
        else { kind = (s + 1 < T.nsteps) ? Q_KIN_FULL : Q_KIN_HALF; off = r - td - tr - tp; }
    } else {
        kind = Q_EXIT;
        s = T.nsteps;
        off = x - te - tk - step * (unsigned long long)T.nsteps;
    }
    // instance: last i with prefix[i] <= off (binary search)
    const int base = (kind == Q_KIN_HALF && s >= 0 ? Q_KIN_FULL : kind) * (T.count + 1);
    int lo = 0, hi = T.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (T.prefix[base + mid] <= off) lo = mid;
        else hi = mid - 1;
    }
    it.kind = kind;
    it.inst = lo;
    it.tile = (int)(off - T.prefix[base + lo]);
    // tiles of this instance in all earlier phases
    const int i = lo;
    const unsigned long long pre = (unsigned long long)qtiles(T, Q_ENTRY, i) + qtiles(T, Q_KIN_HALF, i);
    const unsigned long long per = (unsigned long long)qtiles(T, Q_DENSITY, i) + qtiles(T, Q_KERNEL, i) +
                                   qtiles(T, Q_PHASE, i) + qtiles(T, Q_KIN_FULL, i);
    unsigned long long need;
    if (kind == Q_ENTRY) need = 0;
    else if (s < 0) need = qtiles(T, Q_ENTRY, i);                       // the first half kinetic
    else if (s >= T.nsteps) need = pre + per * (unsigned long long)T.nsteps;   // exit
    else {
        need = pre + per * (unsigned long long)s;
        if (kind == Q_KERNEL || kind == Q_PHASE || kind == Q_KIN_FULL || kind == Q_KIN_HALF)
            need += qtiles(T, Q_DENSITY, i);
        if (kind == Q_PHASE || kind == Q_KIN_FULL || kind == Q_KIN_HALF) need += qtiles(T, Q_KERNEL, i);
        if (kind == Q_KIN_FULL || kind == Q_KIN_HALF) need += qtiles(T, Q_PHASE, i);
    }
    it.need = need;
    return it;
}

}  // namespace gsn
