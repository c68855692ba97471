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
// lconn[(d+1)][n_e] gives each element corner's index into its patch's vertex list. eperm (the
// resident plan only; empty otherwise): the element in each slot of [eoff[k], eoff[k+1]), the
// order in which the workgroup's lanes take them. nshared (resident plan only): patch k's vertex
// list holds first the nshared[k] vertices other patches hold too, then those only it holds.
struct Patches {
  std::vector<int32_t> eoff, voff, verts, eperm, nshared;
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
// than n_blocks patches and no vertex that no element uses. Each patch lists the vertices it
// shares with other patches first (nshared[k] of them), then its interior ones; within each part
// the vertex order, and with move_elements the element slots (eperm; else eperm is the identity),
// are chosen by balance_patch, so neither part is sorted.
isb_status build_resident_patches(int dim, int64_t n_v, int n_bodies, const int64_t* voff, const int64_t* eoff,
                                  const int32_t* T, int n_blocks, int max_verts, bool move_elements, Patches* out,
                                  std::vector<int32_t>* body_patch_off, std::vector<uint8_t>* eligible);


// The patch plan the context builds: at most kPatchMaxElems elements per patch, and as many
// vertices as fit x, p, the FP64 accumulator and the vertex id in kPatchLdsBytes of LDS.
constexpr int kPatchMaxElems = 2048;
constexpr int kPatchLdsBytes = 64 * 1024;  // LDS per patch workgroup (two workgroups per CU)
constexpr int patch_max_verts(int dim) { return kPatchLdsBytes / (3 * dim * (int)sizeof(double) + 4); }

// LDS bank balance of one patch of the resident plan. The kernel's lanes take the patch's element
// slots 64 at a time (one wavefront at one step), and the LDS serves an FP64 access in two passes
// of 32 lanes. A vertex with local id v keeps its FP64 values at byte offsets 8 (D v + c), which
// fall in the pair of 4-byte banks (6 v + 2 c) mod 64 (3D; 4 v + 2 c in 2D): the bank class of v is
// v mod 32 (3D) or v mod 16 (2D), the same for all components. A half-wavefront's LDS atomic or
// gather at corner q of its elements costs about as many cycles as the most lanes that share a
// class (measured on one CU: 8.2 cycles per wavefront FP64 atomic with one lane per class in each
// half, 24.1 at random vertices). On the nk-corner elements tloc[ne][nk] (patch-local
// vertex ids < nv), order[s] receives the element of slot s and newid[v] the new local id of vertex
// v: a greedy grouping of the slots in groups of 32, then a short local search over element swaps
// between groups and exchanges of vertex ids, lowering the sum over groups, corners and classes of
// count squared (and, when elements move, a steep cost on two lanes of a group at one vertex, whose
// atomics serialise outright). On the Kuhn-tet block's 1,536-element patches in wave order the mean
// largest count per half-wavefront falls from about 2.4 to 2.0 (ideal 1). Deterministic.
// With move_elements false the slots keep the elements' order (order is the identity) and only
// the vertex numbering is chosen; with renumber false the numbering is kept (newid is the identity)
// and only the slots are chosen. Vertex ids change only inside a window of consecutive ids (one id
// per class) and never across split: ids below it stay below it.
void balance_patch(int dim, int ne, int nv, const int32_t* tloc, bool move_elements, int split,
                   std::vector<int32_t>* order, std::vector<int32_t>* newid, bool renumber = true);
// balance_patch on every patch of out (n_e elements in all): eperm receives each patch's slots
// (the identity without move_elements), lconn and verts the new vertex numbering
void balance_patches(int dim, int64_t n_e, bool move_elements, Patches* out);
// mean over (group, corner) of the largest class count, for the slots and numbering given
double patch_bank_load(int dim, int ne, const int32_t* tloc, const int32_t* order, const int32_t* newid);

// Element order inside each patch of that plan: first the wavefront groups (64 consecutive
// elements from the patch's first) are packed with distinct vertices per corner slot where
// possible; then balance_patch moves elements between the half-wavefront groups, with the plan's
// vertex numbering (sorted global ids) kept, so that each half-wavefront's corners spread over the
// LDS bank classes, and the packed order stays where that does not lower the largest class counts.
isb_status wave_order(int dim, int64_t n_v, int n_bodies, const int64_t* eoff, const int32_t* T, int64_t* perm);

}  // namespace isb
