// Validation of a problem description (ganmres_config), shared by the
// handle-based entry points and the allocation-free objective.
#pragma once

#include <string>

#include "../../include/ganmres.h"
#include "fft_core.hpp"

namespace gan {

// Grid sizes 2^a 3^b in [4, 1024] (the transforms' radices).
inline bool size_ok(int n) {
    if (n < 4 || n > 1024) return false;
    int r[kMaxRadices];
    return make_radices(n, r) > 0;
}

// Message of the last failure of a call without a handle (ganmres_create,
// ganmres_create_batch, ganmres_eval_objective_noalloc) on this thread; read
// by ganmres_last_error(NULL).
std::string& handle_free_error();

// Empty when c describes a valid problem, else the reason.
inline std::string config_error(const ganmres_config& c) {
    if (c.dim != 2 && c.dim != 3) return "dim must be 2 or 3";
    for (int a = 0; a < c.dim; ++a)
        if (!size_ok(c.n[a])) return "grid sizes must be 2^a 3^b in [4, 1024]";
    if (c.nt < 1) return "nt must be >= 1";
    if (c.nt > 64) return "nt must be <= 64";
    if (!(c.alpha > 0.0)) return "alpha must be > 0";
    if (c.reg_order < 1 || c.reg_order > 3) return "reg_order must be 1..3";
    if (c.model != GANMRES_ADVECTION && c.model != GANMRES_CONTINUITY) return "unknown model";
    if (c.dtype != GANMRES_F32 && c.dtype != GANMRES_F64) return "unknown dtype";
    if (c.incompressible && c.model == GANMRES_CONTINUITY)
        return "the incompressible option applies to the advection model";
    if (c.checkpoint_every < 1) return "checkpoint_every must be >= 1";
    return std::string();
}

}  // namespace gan
