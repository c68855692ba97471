// Test infrastructure only: the resident CG plan builder of isb_host.cpp behind a C entry point, so
// that its invariants can be checked on the CPU. Output arrays are sized by the caller for the
// worst case (one patch per element): eoff, voff [n_e + 1], verts, lconn [(dim + 1) * n_e], eperm
// [n_e], nshared [n_e], body_patch_off [n_bodies + 1], eligible [n_bodies]; counts[0..2] = patches, patch vertices,
// max_nv. emu_patch_balance runs the bank balance of one patch (tloc [ne][dim + 1] local ids < nv)
// and returns the mean largest class count before (slots and ids as given) and after.
#include <cstring>

#include "isb_host.hpp"

extern "C" int emu_resident_plan(int dim, int64_t n_v, int n_bodies, const int64_t* voff, const int64_t* eoff,
                                 const int32_t* T, int n_blocks, int max_verts, int move_elements, int32_t* p_eoff,
                                 int32_t* p_voff, int32_t* p_verts, uint16_t* p_lconn, int32_t* p_eperm,
                                 int32_t* p_nshared, int32_t* body_patch_off, uint8_t* eligible, int32_t* counts) {
  isb::Patches pt;
  std::vector<int32_t> bpo;
  std::vector<uint8_t> ok;
  const isb_status st =
      isb::build_resident_patches(dim, n_v, n_bodies, voff, eoff, T, n_blocks, max_verts, move_elements != 0, &pt,
                                  &bpo, &ok);
  if (st != ISB_OK) return (int)st;
  std::memcpy(p_eoff, pt.eoff.data(), pt.eoff.size() * sizeof(int32_t));
  std::memcpy(p_voff, pt.voff.data(), pt.voff.size() * sizeof(int32_t));
  std::memcpy(p_verts, pt.verts.data(), pt.verts.size() * sizeof(int32_t));
  std::memcpy(p_lconn, pt.lconn.data(), pt.lconn.size() * sizeof(uint16_t));
  std::memcpy(p_eperm, pt.eperm.data(), pt.eperm.size() * sizeof(int32_t));
  std::memcpy(p_nshared, pt.nshared.data(), pt.nshared.size() * sizeof(int32_t));
  std::memcpy(body_patch_off, bpo.data(), bpo.size() * sizeof(int32_t));
  std::memcpy(eligible, ok.data(), ok.size());
  counts[0] = (int32_t)pt.eoff.size() - 1;
  counts[1] = (int32_t)pt.verts.size();
  counts[2] = pt.max_nv;
  return 0;
}

extern "C" void emu_patch_balance(int dim, int ne, int nv, const int32_t* tloc, int move_elements, int32_t* order_out,
                                  int32_t* newid_out, double* loads) {
  std::vector<int32_t> ident_e(ne), ident_v(nv), order, newid;
  for (int e = 0; e < ne; ++e) ident_e[e] = e;
  for (int v = 0; v < nv; ++v) ident_v[v] = v;
  loads[0] = isb::patch_bank_load(dim, ne, tloc, ident_e.data(), ident_v.data());
  isb::balance_patch(dim, ne, nv, tloc, move_elements != 0, nv, &order, &newid);
  loads[1] = isb::patch_bank_load(dim, ne, tloc, order.data(), newid.data());
  std::memcpy(order_out, order.data(), ne * sizeof(int32_t));
  std::memcpy(newid_out, newid.data(), nv * sizeof(int32_t));
}
