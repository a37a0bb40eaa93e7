// Static race check of the factorisation schedule (see race.cpp).
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

}  // namespace d3m
