// Gate matrices and validation (host).
#pragma once

#include <string>

#include "../../include/sv.h"
#include "qv_internal.h"

namespace qv {

bool is_two_qubit_op(int op);

// "" if the gate is valid for an n-qubit state, else the reason.
std::string check_gate(const sv_gate& g, int n);

// True (with the reason) for valid gates this engine does not implement.
bool unsupported_gate(const sv_gate& g, std::string* why);

// Matrix (or diagonal) of a validated gate, in FP64.
HostGate build_gate(const sv_gate& g);

// Sweep form of a gate: a diagonal with ones on a bit-0 half becomes a
// controlled diagonal on the rest, so its sweep touches only that part.
HostGate sweep_form(const HostGate& g);

}  // namespace qv
