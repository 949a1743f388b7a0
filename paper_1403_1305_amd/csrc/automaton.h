// automaton.h -- the library's automaton object and error reporting (internal).
#pragma once

#include <string>
#include <vector>

#include "../../include/ac.h"
#include "machine.h"
#include "scan.h"

struct ac_automaton {
    acm::Machine m;
    acm::DeviceMachine dm;
    bool on_device = false;
    int device = -1;
    uint32_t placement = AC_PLACE_GLOBAL;  // resolved default for scans
    std::vector<void *> allocations;
};

namespace acm {
// Record `msg` as this thread's last error and return `code`.
int set_error(int code, const std::string &msg);

// The matcher AC_ALGO_AUTO runs: the gated failure-less scan where its gate
// passes few enough start positions that walking them costs less than the
// DFA's lookup per byte, else the DFA (the failure-less scan without DFA).
constexpr double kGateAutoPass = 0.05;
inline uint32_t auto_algo(const ac_automaton *a) {
    if ((a->dm.gate_bits || a->dm.qg_bits) && a->m.gate_pass <= kGateAutoPass) return AC_ALGO_GATED;
    return a->m.goto_only ? AC_ALGO_PFAC : AC_ALGO_DFA;
}
}  // namespace acm
