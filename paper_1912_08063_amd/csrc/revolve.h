// revolve.h -- binomial checkpointing schedules (host C++).
//
// Reversal problem: forward states 0..l are produced by l leapfrog steps; the
// adjoint sweep needs states l-1, l-2, ..., 1 in that order (state 0 is the
// zero field and never needs a slot).  With s snapshot slots (the free zero
// state counts as one more), the minimal number of forward steps is the
// Griewank-Walther binomial bound  t(l, s) = r l - beta(s + 1, r - 1),
// beta(s, r) = C(s + r, s), r the least integer with beta(s, r) >= l.
#pragma once
#include <stdint.h>

#include <vector>

namespace fwi {

enum RevolveOp { OP_ADVANCE = 1, OP_TAKESHOT = 2, OP_RESTORE = 3, OP_ADJOINT = 4, OP_RESTART = 5 };

struct Action {
    int32_t op;
    int32_t arg;   // ADVANCE: target time; TAKESHOT/RESTORE: slot; ADJOINT: time
};

// beta(s, r) = C(s + r, s), saturating at 2^62.
int64_t revolve_beta(int64_t s, int64_t r);

// Minimal forward steps to reverse l steps with s snapshots (s >= 1 counts
// the snapshot that holds the starting state).
int64_t revolve_cost(int64_t l, int64_t s);

// Schedule for the adjoint of nsteps forward steps with `slots` physical
// snapshot slots plus the free zero state.  *forward_steps receives the
// number of forward steps the schedule performs, not counting the extra step
// from nsteps-1 to nsteps the recording sweep makes.
std::vector<Action> revolve_schedule(int32_t nsteps, int32_t slots, int64_t *forward_steps);

}  // namespace fwi
