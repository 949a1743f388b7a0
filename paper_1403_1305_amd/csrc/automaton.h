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
}  // namespace acm
