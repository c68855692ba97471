// Test infrastructure only: the resident CG plan builder of isb_host.cpp behind a C entry point, so
// that its invariants can be checked on the CPU. Output arrays are sized by the caller for the
// worst case (one patch per element): eoff, voff [n_e + 1], verts, lconn [(dim + 1) * n_e],
// body_patch_off [n_bodies + 1], eligible [n_bodies]; counts[0..2] = patches, patch vertices, max_nv.
#include <cstring>

#include "isb_host.hpp"

extern "C" int emu_resident_plan(int dim, int64_t n_v, int n_bodies, const int64_t* voff, const int64_t* eoff,
                                 const int32_t* T, int n_blocks, int max_verts, int32_t* p_eoff, int32_t* p_voff,
                                 int32_t* p_verts, uint16_t* p_lconn, int32_t* body_patch_off, uint8_t* eligible,
                                 int32_t* counts) {
  isb::Patches pt;
  std::vector<int32_t> bpo;
  std::vector<uint8_t> ok;
  const isb_status st =
      isb::build_resident_patches(dim, n_v, n_bodies, voff, eoff, T, n_blocks, max_verts, &pt, &bpo, &ok);
  if (st != ISB_OK) return (int)st;
  std::memcpy(p_eoff, pt.eoff.data(), pt.eoff.size() * sizeof(int32_t));
  std::memcpy(p_voff, pt.voff.data(), pt.voff.size() * sizeof(int32_t));
  std::memcpy(p_verts, pt.verts.data(), pt.verts.size() * sizeof(int32_t));
  std::memcpy(p_lconn, pt.lconn.data(), pt.lconn.size() * sizeof(uint16_t));
  std::memcpy(body_patch_off, bpo.data(), bpo.size() * sizeof(int32_t));
  std::memcpy(eligible, ok.data(), ok.size());
  counts[0] = (int32_t)pt.eoff.size() - 1;
  counts[1] = (int32_t)pt.verts.size();
  counts[2] = pt.max_nv;
  return 0;
}
