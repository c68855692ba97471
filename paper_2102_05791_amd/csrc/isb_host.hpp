// Host-only helpers shared by the C-ABI implementation.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/isb.h"

namespace isb {

isb_status fail(isb_status st, const std::string& msg);
void clear_error();
const char* last_error();
isb_status validate_mesh(int dim, int64_t n_v, const double* X, int64_t n_e, const int32_t* T, int32_t n_bodies,
                         const int64_t* voff, const int64_t* eoff);
isb_status colour_elements(int dim, int64_t n_v, int64_t n_e, const int32_t* T, int32_t* colour, int32_t* n_colours);

// Element patches for the LDS-staged scatter: patch k holds the consecutive elements
// [eoff[k], eoff[k+1]) of one body and the sorted distinct vertices verts[voff[k] .. voff[k+1]);
// lconn[(d+1)][n_e] gives each element corner's index into its patch's vertex list.
struct Patches {
  std::vector<int32_t> eoff, voff, verts;
  std::vector<uint16_t> lconn;
  int max_nv = 0;
};
// per_body: patches a body is cut into when that leaves at least 256 elements in each (rounded
// to whole 64-element wavefronts); max_elems and max_verts cap every patch.
isb_status build_patches(int dim, int64_t n_v, int n_bodies, const int64_t* eoff, const int32_t* T,
                         int max_elems, int max_verts, Patches* out, int per_body = 1024);

// The resident CG solver's plan: each body cut into at most n_blocks patches (one per resident
// workgroup) of at most max_verts vertices. Each vertex is owned by the first patch that holds it;
// verts stores v for an owned vertex and ~v (negative) for one that another patch owns. Body b's
// patches are [body_patch_off[b], body_patch_off[b + 1]); eligible[b] when it has elements, no more
// than n_blocks patches and no vertex that no element uses.
isb_status build_resident_patches(int dim, int64_t n_v, int n_bodies, const int64_t* voff, const int64_t* eoff,
                                  const int32_t* T, int n_blocks, int max_verts, Patches* out,
                                  std::vector<int32_t>* body_patch_off, std::vector<uint8_t>* eligible);


// The patch plan the context builds: at most kPatchMaxElems elements per patch, and as many
// vertices as fit x, p, the FP64 accumulator and the vertex id in kPatchLdsBytes of LDS.
constexpr int kPatchMaxElems = 2048;
constexpr int kPatchLdsBytes = 64 * 1024;  // LDS per patch workgroup (two workgroups per CU)
constexpr int patch_max_verts(int dim) { return kPatchLdsBytes / (3 * dim * (int)sizeof(double) + 4); }

// Element order inside each patch of that plan in which the wavefront groups (64 consecutive
// elements from the patch's first) hold distinct vertices per corner slot where possible.
isb_status wave_order(int dim, int64_t n_v, int n_bodies, const int64_t* eoff, const int32_t* T, int64_t* perm);

}  // namespace isb
