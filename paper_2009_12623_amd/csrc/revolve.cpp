// Binomial checkpoint schedule (paper Sec. 1.3 "Checkpointing", Fig. 2;
// the optimal schedules of Revolve, which the paper cites).
//
// The reverse sweep needs forward states x_N .. x_1 (x_k = (u^k, u^{k-1}));
// x_0 = 0 is free.  With s slots the least number of forward steps is
//   T(n, 0) = n(n+1)/2,  T(0, s) = 0,
//   T(n, s) = min_j [ j + T(n-j, s-1) + T(j-1, s) ],
// equal to the classic binomial count for n+1 steps and s+1 snapshots:
//   t l - C(c + t, t - 1),  l = n + 1, c = s + 1,  t least with C(c+t, c) >= l.
// The split taken is the largest j reaching the minimum.  Slots form a
// stack; a restore is emitted only when the working state differs.
#include <cstdint>
#include <vector>

#include "../../include/fwigrad.h"

namespace fwi {

namespace {

long long steps_min(long long n, long long s)
{
    if (n <= 0) return 0;
    if (s <= 0) return n * (n + 1) / 2;
    if (s >= n) return n;                       // every state stored
    const long long l = n + 1, c = s + 1;
    // C(c+t, c) for t = 0, 1, ... until it reaches l
    __int128 cb = 1;
    long long t = 0;
    while (cb < l) {
        ++t;
        cb = cb * (c + t) / t;
    }
    const __int128 cb1 = cb * t / (c + 1);      // C(c+t, c+1) = C(c+t, t-1)
    return (long long)((__int128)t * l - cb1);
}

struct Planner {
    std::vector<fwi_action> acts;
    int work = 0;
    int depth = 0;

    void emit(int op, int a, int b) { acts.push_back(fwi_action{op, a, b}); }

    void ensure(int k, int slot)
    {
        if (work != k) {
            emit(FWI_RESTORE, slot, k);
            work = k;
        }
    }

    static int split(int n, int s)
    {
        long long best = -1;
        int arg = 1;
        for (int j = 1; j <= n; ++j) {
            long long v = j + steps_min(n - j, s - 1) + steps_min(j - 1, s);
            if (best < 0 || v <= best) {
                best = v;
                arg = j;
            }
        }
        return arg;
    }

    // reverse states b .. a+1; x_a is in `slot_a` (-1: the zero state)
    void run(int a, int b, int s, int slot_a)
    {
        while (b > a) {
            ensure(a, slot_a);
            if (s == 0) {
                emit(FWI_ADVANCE, a, b);
                work = b;
                emit(FWI_REVERSE, b, 0);
                --b;
                continue;
            }
            const int m = a + split(b - a, s);
            emit(FWI_ADVANCE, a, m);
            work = m;
            if (m == b) {
                emit(FWI_REVERSE, b, 0);
                --b;
                continue;
            }
            const int slot = depth++;
            emit(FWI_TAKESHOT, slot, m);
            run(m, b, s - 1, slot);
            ensure(m, slot);
            emit(FWI_REVERSE, m, 0);
            emit(FWI_FREE, slot, 0);
            --depth;
            b = m - 1;
        }
    }
};

}  // namespace

std::vector<fwi_action> revolve_plan(int nsteps, int nslots)
{
    Planner p;
    p.run(0, nsteps, nslots < nsteps ? nslots : nsteps, -1);
    return std::move(p.acts);
}

long long revolve_min_steps(int nsteps, int nslots)
{
    return steps_min(nsteps, nslots < nsteps ? nslots : nsteps);
}

}  // namespace fwi
