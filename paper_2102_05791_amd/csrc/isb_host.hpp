// Host-only helpers shared by the C-ABI implementation.
#pragma once

#include <stdint.h>

#include <string>

#include "../../include/isb.h"

namespace isb {

isb_status fail(isb_status st, const std::string& msg);
void clear_error();
const char* last_error();
isb_status validate_mesh(int dim, int64_t n_v, const double* X, int64_t n_e, const int32_t* T, int32_t n_bodies,
                         const int64_t* voff, const int64_t* eoff);
isb_status colour_elements(int dim, int64_t n_v, int64_t n_e, const int32_t* T, int32_t* colour, int32_t* n_colours);

}  // namespace isb
