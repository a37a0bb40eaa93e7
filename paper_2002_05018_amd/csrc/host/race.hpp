// Static race check of the factorisation schedule (race.cpp) and simulation
// of the work-queue solve sweeps (chain_sim.cpp).
#pragma once

#include <string>

#include "plan.hpp"

namespace d3m {

// The launch shapes that decide the streams and waits of the factor sweeps.
struct ScheduleModel {
    int64_t lookahead_tasks = 0;  // 0: the library default
    int side_early = 0;
    int k_overlap = 0;
    bool one_stream_k = false;    // the K phase on the caller's stream only
    bool drop_waits = false;      // a planted mistake for tests of the check: no
                                  // stream waits for earlier side-stream updates
};

// Number of unordered conflicting tile accesses of one factorisation (0: the
// schedule is race-free); the first ones are described in report.
int64_t check_factor_schedule(const Plan &pl, const ScheduleModel &m, std::string &report);

// Simulates the work-queue form of the two K solve sweeps (chain_sim.cpp):
// workers take items from one counter and wait on write counts as the kernel
// does, under pseudo-random interleavings, for 1 and 2 column blocks and
// several worker counts.  Returns the number of violations (an item that
// sees a tile with other writes than the sequential order gives it, or a
// stalled queue), -1 when the plan has no such form (reason in report).
// drop_wait leaves out each item's first wait (a planted mistake for tests).
int64_t check_solve_chain(const Plan &pl, bool drop_wait, std::string &report);

}  // namespace d3m
