// revolve.cpp -- binomial checkpointing (Griewank & Walther's "revolve"),
// written as a recursion over the optimal split point.
//
// rev(a, b, s): state a is available (restorable), states b-1 .. a must be
// visited in that order, s snapshots may be used (the one holding a
// included).  With one snapshot every visit re-advances from a; otherwise
// advance to a + m, store it, reverse [a+m, b) with s-1 snapshots, release
// the slot and reverse [a, a+m) with s.  The split m minimises
//     m + t(l - m, s - 1) + t(m, s)   (l = b - a),
// evaluated with the closed-form cost t, so the schedule attains t(l, s).
#include "revolve.h"

#include <algorithm>

namespace fwi {

int64_t revolve_beta(int64_t s, int64_t r)
{
    if (r < 0 || s < 0) return 0;
    const int64_t cap = int64_t(1) << 62;
    int64_t b = 1;   // C(s + i, i) for i = 0..r
    for (int64_t i = 1; i <= r; ++i) {
        // C(s+i, i) = C(s+i-1, i-1) * (s+i) / i, exact in integers
        const __int128 t = (__int128)b * (s + i) / i;
        if (t >= cap) return cap;
        b = (int64_t)t;
    }
    return b;
}

int64_t revolve_cost(int64_t l, int64_t s)
{
    if (l <= 1) return 0;
    if (s <= 1) return l * (l - 1) / 2;
    int64_t r = 0;
    while (revolve_beta(s, r) < l) ++r;
    return r * l - revolve_beta(s + 1, r - 1);
}

namespace {

struct Gen {
    std::vector<Action> out;
    std::vector<int32_t> slot_busy;
    int32_t cur = 0;
    int64_t steps = 0;

    void emit(int32_t op, int32_t arg) { out.push_back(Action{op, arg}); }

    void restore(int32_t a, int32_t slot)
    {
        if (cur == a) return;
        if (a == 0) emit(OP_RESTART, 0); else emit(OP_RESTORE, slot);
        cur = a;
    }
    void advance(int32_t to)
    {
        if (to > cur) { emit(OP_ADVANCE, to); steps += to - cur; cur = to; }
    }
    void visit(int32_t k) { if (k >= 1) emit(OP_ADJOINT, k); }

    int32_t take_slot()
    {
        for (size_t i = 0; i < slot_busy.size(); ++i)
            if (!slot_busy[i]) { slot_busy[i] = 1; return (int32_t)i; }
        return -1;   // unreachable: the recursion never holds more than `slots`
    }

    static int32_t best_split(int64_t l, int64_t s)
    {
        // enough snapshots to store every state: one step per snapshot
        if (revolve_cost(l, s) == l - 1) return 1;
        int64_t best = -1, bm = 1;
        for (int64_t m = 1; m < l; ++m) {
            const int64_t c = m + revolve_cost(l - m, s - 1) + revolve_cost(m, s);
            if (best < 0 || c < best) { best = c; bm = m; }
        }
        return (int32_t)bm;
    }

    void rev(int32_t a, int32_t b, int64_t s, int32_t slot_a)
    {
        if (b - a <= 0) return;
        if (b - a == 1) { restore(a, slot_a); visit(a); return; }
        if (s <= 1) {
            for (int32_t k = b - 1; k >= a; --k) { restore(a, slot_a); advance(k); visit(k); }
            return;
        }
        const int32_t m = a + best_split(b - a, s);
        restore(a, slot_a);
        advance(m);
        const int32_t sl = take_slot();
        emit(OP_TAKESHOT, sl);
        rev(m, b, s - 1, sl);
        slot_busy[sl] = 0;
        rev(a, m, s, slot_a);
    }
};

}  // namespace

std::vector<Action> revolve_schedule(int32_t nsteps, int32_t slots, int64_t *forward_steps)
{
    Gen g;
    g.slot_busy.assign(std::max(slots, 0), 0);
    g.rev(0, nsteps, (int64_t)std::max(slots, 0) + 1, -1);
    if (forward_steps) *forward_steps = g.steps;
    return g.out;
}

}  // namespace fwi
