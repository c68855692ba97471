// Host-only parts of libisb: mesh validation, element colouring, error reporting.
// Nothing here touches the GPU, so these entry points work on a machine without one.
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/isb.h"
#include "isb_host.hpp"

namespace isb {

static thread_local std::string g_last_error;

isb_status fail(isb_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

void clear_error() { g_last_error.clear(); }

const char* last_error() { return g_last_error.c_str(); }

// det of the edge matrix [x_1 - x_0, ..., x_d - x_0]
static double edge_det(int dim, const double* X, const int32_t* t) {
  double e[3][3];
  for (int j = 0; j < dim; ++j)
    for (int c = 0; c < dim; ++c) e[c][j] = X[(int64_t)t[j + 1] * dim + c] - X[(int64_t)t[0] * dim + c];
  if (dim == 2) return e[0][0] * e[1][1] - e[0][1] * e[1][0];
  return e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
         e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
}

isb_status validate_mesh(int dim, int64_t n_v, const double* X, int64_t n_e, const int32_t* T, int32_t n_bodies,
                         const int64_t* voff, const int64_t* eoff) {
  if (dim != 2 && dim != 3) return fail(ISB_E_ARG, "dim must be 2 or 3");
  if (n_v <= 0 || n_e <= 0 || n_bodies <= 0) return fail(ISB_E_ARG, "empty mesh");
  if (!X || !T || !voff || !eoff) return fail(ISB_E_ARG, "NULL mesh array");
  if (n_v > INT32_MAX / 4 || n_e > INT32_MAX / 16) return fail(ISB_E_ARG, "mesh too large for 32-bit indexing");
  if (voff[0] != 0 || eoff[0] != 0 || voff[n_bodies] != n_v || eoff[n_bodies] != n_e)
    return fail(ISB_E_MESH, "body offsets must start at 0 and end at n_v / n_e");
  for (int32_t b = 0; b < n_bodies; ++b) {
    if (voff[b + 1] <= voff[b] || eoff[b + 1] <= eoff[b])
      return fail(ISB_E_MESH, "body " + std::to_string(b) + " has no vertices or no elements");
  }
  for (int64_t i = 0; i < n_v * dim; ++i)
    if (!std::isfinite(X[i])) return fail(ISB_E_MESH, "non-finite rest position");
  for (int32_t b = 0; b < n_bodies; ++b) {
    for (int64_t e = eoff[b]; e < eoff[b + 1]; ++e) {
      const int32_t* t = T + e * (dim + 1);
      for (int k = 0; k <= dim; ++k) {
        if (t[k] < voff[b] || t[k] >= voff[b + 1])
          return fail(ISB_E_MESH, "element " + std::to_string(e) + " references vertex " + std::to_string(t[k]) +
                                      " outside body " + std::to_string(b));
        for (int j = 0; j < k; ++j)
          if (t[j] == t[k]) return fail(ISB_E_MESH, "element " + std::to_string(e) + " repeats a vertex");
      }
      const double det = edge_det(dim, X, t);
      if (!(det > 0.0))
        return fail(ISB_E_MESH, "element " + std::to_string(e) + " has non-positive rest volume (det " +
                                    std::to_string(det) + ")");
    }
  }
  return ISB_OK;
}

isb_status colour_elements(int dim, int64_t n_v, int64_t n_e, const int32_t* T, int32_t* colour,
                           int32_t* n_colours) {
  // greedy first-fit in element order; a 64-bit mask per vertex holds the colours of its elements
  std::vector<uint64_t> used((size_t)n_v, 0);
  int32_t nc = 0;
  for (int64_t e = 0; e < n_e; ++e) {
    const int32_t* t = T + e * (dim + 1);
    uint64_t m = 0;
    for (int k = 0; k <= dim; ++k) {
      if (t[k] < 0 || t[k] >= n_v) return fail(ISB_E_MESH, "vertex index out of range in colouring");
      m |= used[t[k]];
    }
    if (m == ~0ull) return fail(ISB_E_MESH, "element colouring needs more than 64 colours");
    int c = 0;
    while (m & (1ull << c)) ++c;
    colour[e] = c;
    for (int k = 0; k <= dim; ++k) used[t[k]] |= (1ull << c);
    if (c + 1 > nc) nc = c + 1;
  }
  *n_colours = nc;
  return ISB_OK;
}

isb_status build_patches(int dim, int64_t n_v, int n_bodies, const int64_t* eoff, const int32_t* T,
                         int max_elems, int max_verts, Patches* out, int per_body) {
  const int64_t n_e = eoff[n_bodies];
  out->eoff.assign(1, 0);
  out->voff.assign(1, 0);
  out->verts.clear();
  out->lconn.assign((size_t)(dim + 1) * (size_t)n_e, 0);
  out->max_nv = 0;
  // mark[v] = last patch that took vertex v, so that each corner is counted in O(1)
  std::vector<int32_t> mark((size_t)n_v, -1);
  std::vector<int32_t> ids;
  int32_t patch = 0;
  for (int b = 0; b < n_bodies; ++b) {
    // per_body patches per body when it is large enough (a thousand fill the GPU in one launch);
    // a whole number of 64-element wavefronts, so that every wavefront of a full patch is full
    const int64_t ne_b = eoff[b + 1] - eoff[b];
    const int64_t per = ((ne_b + per_body - 1) / per_body + 63) / 64 * 64;
    const int64_t me = std::min<int64_t>(max_elems, std::max<int64_t>(256, per));
    int64_t e = eoff[b];
    while (e < eoff[b + 1]) {
      const int64_t start = e;
      ids.clear();
      while (e < eoff[b + 1] && e - start < me) {
        const int32_t* t = T + e * (dim + 1);
        int fresh = 0;
        for (int k = 0; k <= dim; ++k) fresh += mark[t[k]] != patch;
        if ((int64_t)ids.size() + fresh > max_verts) break;
        for (int k = 0; k <= dim; ++k)
          if (mark[t[k]] != patch) {
            mark[t[k]] = patch;
            ids.push_back(t[k]);
          }
        ++e;
      }
      if (e == start) return fail(ISB_E_MESH, "patch builder: one element exceeds the vertex budget");
      std::sort(ids.begin(), ids.end());
      for (int64_t f = start; f < e; ++f)
        for (int k = 0; k <= dim; ++k) {
          const int32_t g = T[f * (dim + 1) + k];
          const auto it = std::lower_bound(ids.begin(), ids.end(), g);
          out->lconn[(size_t)k * n_e + f] = (uint16_t)(it - ids.begin());
        }
      out->verts.insert(out->verts.end(), ids.begin(), ids.end());
      out->eoff.push_back((int32_t)e);
      out->voff.push_back((int32_t)out->verts.size());
      out->max_nv = std::max<int>(out->max_nv, (int)ids.size());
      ++patch;
    }
  }
  return ISB_OK;
}


// ---- LDS bank balance of a resident patch (see isb_host.hpp) ----
namespace {

constexpr int kLanes = 32;  // lanes the LDS serves together in one FP64 pass: half a wavefront

// splitmix64: a small deterministic generator for the local search
struct Mix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  int below(int n) { return (int)(next() % (uint64_t)n); }
};

int bank_classes(int dim) { return dim == 3 ? 32 : 16; }

}  // namespace

void balance_patch(int dim, int ne, int nv, const int32_t* tloc, bool move_elements, int split,
                   std::vector<int32_t>* order, std::vector<int32_t>* newid, bool renumber) {
  const int nk = dim + 1, nc = bank_classes(dim);
  const int ng = (ne + kLanes - 1) / kLanes;
  // the change of the sum of squared counts when one count goes from c to c + 1 or c - 1
  auto up = [](int64_t c) { return 2 * c + 1; };
  auto down = [](int64_t c) { return -2 * c + 1; };
  order->resize(ne);
  newid->resize(nv);
  for (int v = 0; v < nv; ++v) (*newid)[v] = v;
  if (ne == 0) return;
  std::vector<int32_t>& id = *newid;
  // cnt[(g * nk + q) * nc + class]: lanes of group g whose corner q has that class; dup[(g * nk +
  // q) * nv + v]: lanes of group g whose corner q is vertex v. Two lanes at one vertex serialise
  // their atomics outright, so the element moves weigh a repeated vertex kDup times a class clash.
  constexpr int64_t kDup = 16;
  std::vector<int32_t> cnt((size_t)ng * nk * nc, 0);
  std::vector<int32_t> dup(move_elements ? (size_t)ng * nk * nv : 0, 0);
  std::vector<int32_t> grp(ne, -1), fill(ng, 0), cap(ng, kLanes);
  cap[ng - 1] = ne - (ng - 1) * kLanes;
  auto at = [&](int g, int q, int v) -> int32_t& { return cnt[((size_t)g * nk + q) * nc + id[v] % nc]; };
  auto dv = [&](int g, int q, int v) -> int32_t& { return dup[((size_t)g * nk + q) * nv + v]; };
  // greedy: each element to the group with room where its corners' classes are least used (in
  // slot order when the elements stay where they are)
  for (int e = 0; e < ne; ++e) {
    const int32_t* t = tloc + (size_t)e * nk;
    int best = move_elements ? -1 : e / kLanes;
    int64_t bc = 0;
    for (int g = 0; g < ng && move_elements; ++g) {
      if (fill[g] >= cap[g]) continue;
      int64_t c = 0;
      for (int q = 0; q < nk; ++q) c += up(at(g, q, t[q])) + kDup * up(dv(g, q, t[q]));
      if (best < 0 || c < bc) {
        best = g;
        bc = c;
      }
    }
    grp[e] = best;
    ++fill[best];
    for (int q = 0; q < nk; ++q) {
      ++at(best, q, t[q]);
      if (move_elements) ++dv(best, q, t[q]);
    }
  }
  // incidences of each vertex: (element, corner)
  std::vector<int32_t> ioff(nv + 1, 0), inc((size_t)ne * nk);
  for (int e = 0; e < ne; ++e)
    for (int q = 0; q < nk; ++q) ++ioff[tloc[(size_t)e * nk + q] + 1];
  for (int v = 0; v < nv; ++v) ioff[v + 1] += ioff[v];
  {
    std::vector<int32_t> pos(ioff.begin(), ioff.end() - 1);
    for (int e = 0; e < ne; ++e)
      for (int q = 0; q < nk; ++q) inc[pos[tloc[(size_t)e * nk + q]]++] = e * nk + q;
  }
  Mix rng{0x51A7E5EEDull + (uint64_t)ne * 131 + (uint64_t)nv};
  std::vector<int32_t> pos_of(nv);  // the vertex holding each local id
  for (int v = 0; v < nv; ++v) pos_of[id[v]] = v;
  for (int round = 0; round < 2; ++round) {
    // element swaps between two groups
    if (ng > 1 && move_elements)
      for (int it = 0; it < 4 * ne; ++it) {
        const int a = rng.below(ne), b = rng.below(ne);
        const int ga = grp[a], gb = grp[b];
        if (ga == gb) continue;
        const int32_t *ta = tloc + (size_t)a * nk, *tb = tloc + (size_t)b * nk;
        int64_t d = 0;
        for (int q = 0; q < nk; ++q) {
          if (ta[q] != tb[q])
            d += kDup * (down(dv(ga, q, ta[q])) + up(dv(gb, q, ta[q])) + down(dv(gb, q, tb[q])) + up(dv(ga, q, tb[q])));
          const int ca = id[ta[q]] % nc, cb = id[tb[q]] % nc;
          if (ca == cb) continue;
          // a leaves ga and enters gb; b leaves gb and enters ga
          d += down(cnt[((size_t)ga * nk + q) * nc + ca]) + up(cnt[((size_t)gb * nk + q) * nc + ca]);
          d += down(cnt[((size_t)gb * nk + q) * nc + cb]) + up(cnt[((size_t)ga * nk + q) * nc + cb]);
        }
        if (d >= 0) continue;
        for (int q = 0; q < nk; ++q) {
          --at(ga, q, ta[q]);
          ++at(gb, q, ta[q]);
          --at(gb, q, tb[q]);
          ++at(ga, q, tb[q]);
          --dv(ga, q, ta[q]);
          ++dv(gb, q, ta[q]);
          --dv(gb, q, tb[q]);
          ++dv(ga, q, tb[q]);
        }
        grp[a] = gb;
        grp[b] = ga;
      }
    // exchanges of two vertices' local ids (their classes), only within a window of nc consecutive
    // ids: the patch's per-DOF loops walk the ids in order, so each wavefront's global loads and
    // stores then stay on the cache lines of the sorted order
    for (int it = 0; renumber && it < 4 * nv; ++it) {
      const int u = rng.below(nv);
      const int lo = std::max(id[u] / nc * nc, id[u] < split ? 0 : split);
      const int hi = std::min(id[u] / nc * nc + nc, id[u] < split ? split : nv);
      const int w = pos_of[lo + rng.below(hi - lo)];
      const int cu = id[u] % nc, cw = id[w] % nc;
      if (cu == cw) continue;
      // moving u's incidences from class cu to cw and w's from cw to cu; where u and w share a
      // (group, corner) the two moves cancel, so apply them one at a time to the counts
      int64_t d = 0;
      for (int k = ioff[u]; k < ioff[u + 1]; ++k) {
        const int e = inc[k] / nk, q = inc[k] % nk;
        int32_t* c = &cnt[((size_t)grp[e] * nk + q) * nc];
        d += down(c[cu]);
        --c[cu];
        d += up(c[cw]);
        ++c[cw];
      }
      for (int k = ioff[w]; k < ioff[w + 1]; ++k) {
        const int e = inc[k] / nk, q = inc[k] % nk;
        int32_t* c = &cnt[((size_t)grp[e] * nk + q) * nc];
        d += down(c[cw]);
        --c[cw];
        d += up(c[cu]);
        ++c[cu];
      }
      if (d < 0) {
        std::swap(id[u], id[w]);
        pos_of[id[u]] = u;
        pos_of[id[w]] = w;
        continue;
      }
      // undo
      for (int k = ioff[w]; k < ioff[w + 1]; ++k) {
        const int e = inc[k] / nk, q = inc[k] % nk;
        int32_t* c = &cnt[((size_t)grp[e] * nk + q) * nc];
        --c[cu];
        ++c[cw];
      }
      for (int k = ioff[u]; k < ioff[u + 1]; ++k) {
        const int e = inc[k] / nk, q = inc[k] % nk;
        int32_t* c = &cnt[((size_t)grp[e] * nk + q) * nc];
        --c[cw];
        ++c[cu];
      }
    }
  }
  // slots: group by group, each in the original element order
  std::fill(fill.begin(), fill.end(), 0);
  for (int e = 0; e < ne; ++e) {
    const int g = grp[e];
    (*order)[(size_t)g * kLanes + fill[g]++] = e;
  }
  // the search lowers the sum of squared counts, not always the largest count: keep the layout it
  // started from unless the largest counts fall
  std::vector<int32_t> ident_e(ne), ident_v(nv);
  for (int e = 0; e < ne; ++e) ident_e[e] = e;
  for (int v = 0; v < nv; ++v) ident_v[v] = v;
  if (patch_bank_load(dim, ne, tloc, order->data(), id.data()) >=
      patch_bank_load(dim, ne, tloc, ident_e.data(), ident_v.data())) {
    *order = ident_e;
    id = ident_v;
  }
}

double patch_bank_load(int dim, int ne, const int32_t* tloc, const int32_t* order, const int32_t* newid) {
  const int nk = dim + 1, nc = bank_classes(dim);
  const int ng = (ne + kLanes - 1) / kLanes;
  if (ng == 0) return 0.0;
  double tot = 0.0;
  std::vector<int> c(nc);
  for (int g = 0; g < ng; ++g)
    for (int q = 0; q < nk; ++q) {
      std::fill(c.begin(), c.end(), 0);
      int mx = 0;
      for (int s = g * kLanes; s < std::min(ne, (g + 1) * kLanes); ++s)
        mx = std::max(mx, ++c[newid[tloc[(size_t)order[s] * nk + q]] % nc]);
      tot += mx;
    }
  return tot / (ng * nk);
}

void balance_patches(int dim, int64_t n_e, bool move_elements, Patches* out) {
  const int nk = dim + 1;
  const bool split = out->nshared.size() + 1 == out->eoff.size();
  out->eperm.resize((size_t)n_e);
  std::vector<int32_t> tloc, order, newid, vnew;
  for (size_t k = 0; k + 1 < out->eoff.size(); ++k) {
    const int e0 = out->eoff[k], ne = out->eoff[k + 1] - e0;
    const int v0 = out->voff[k], nv = out->voff[k + 1] - v0;
    tloc.resize((size_t)ne * nk);
    for (int e = 0; e < ne; ++e)
      for (int q = 0; q < nk; ++q) tloc[(size_t)e * nk + q] = out->lconn[(size_t)q * n_e + e0 + e];
    balance_patch(dim, ne, nv, tloc.data(), move_elements, split ? out->nshared[k] : nv, &order, &newid);
    for (int s = 0; s < ne; ++s) out->eperm[(size_t)e0 + s] = e0 + order[s];
    for (int e = 0; e < ne; ++e)
      for (int q = 0; q < nk; ++q) out->lconn[(size_t)q * n_e + e0 + e] = (uint16_t)newid[tloc[(size_t)e * nk + q]];
    vnew.resize(nv);
    for (int v = 0; v < nv; ++v) vnew[newid[v]] = out->verts[(size_t)v0 + v];
    std::copy(vnew.begin(), vnew.end(), out->verts.begin() + v0);
  }
}

isb_status build_resident_patches(int dim, int64_t n_v, int n_bodies, const int64_t* voff, const int64_t* eoff,
                                  const int32_t* T, int n_blocks, int max_verts, bool move_elements, Patches* out,
                                  std::vector<int32_t>* body_patch_off, std::vector<uint8_t>* eligible) {
  if (n_blocks < 1) return fail(ISB_E_ARG, "resident plan: no workgroups");
  const isb_status st = build_patches(dim, n_v, n_bodies, eoff, T, 1 << 30, max_verts, out, n_blocks);
  if (st != ISB_OK) return st;
  // each patch's vertices: those other patches hold too first, then its interior ones (each part in
  // the sorted order), so that the kernel's per-DOF loops meet the interior DOFs in whole wavefronts
  {
    std::vector<uint8_t> holders((size_t)n_v, 0);
    for (const int32_t v : out->verts) holders[v] = (uint8_t)std::min(2, holders[v] + 1);
    const int np = (int)out->eoff.size() - 1;
    const int nk = dim + 1;
    const int64_t n_e = eoff[n_bodies];
    out->nshared.assign(np, 0);
    std::vector<int32_t> ids, newid;
    for (int k = 0; k < np; ++k) {
      const int v0 = out->voff[k], nv = out->voff[k + 1] - v0;
      ids.assign(out->verts.begin() + v0, out->verts.begin() + v0 + nv);
      newid.resize(nv);
      int ns = 0;
      for (int v = 0; v < nv; ++v) ns += holders[ids[v]] > 1;
      int a = 0, b = ns;
      for (int v = 0; v < nv; ++v) newid[v] = holders[ids[v]] > 1 ? a++ : b++;
      for (int v = 0; v < nv; ++v) out->verts[(size_t)v0 + newid[v]] = ids[v];
      for (int e = out->eoff[k]; e < out->eoff[k + 1]; ++e)
        for (int q = 0; q < nk; ++q) {
          uint16_t& l = out->lconn[(size_t)q * n_e + e];
          l = (uint16_t)newid[l];
        }
      out->nshared[k] = ns;
    }
  }
  balance_patches(dim, eoff[n_bodies], move_elements, out);
  std::vector<uint8_t> owned((size_t)n_v, 0);
  for (size_t i = 0; i < out->verts.size(); ++i) {
    const int32_t v = out->verts[i];
    if (owned[v])
      out->verts[i] = ~v;
    else
      owned[v] = 1;
  }
  // patches of body b: those whose first element lies in it (a patch never spans two bodies)
  const int np = (int)out->eoff.size() - 1;
  body_patch_off->assign((size_t)n_bodies + 1, 0);
  eligible->assign((size_t)n_bodies, 0);
  int k = 0;
  for (int b = 0; b < n_bodies; ++b) {
    (*body_patch_off)[b] = k;
    while (k < np && out->eoff[k] < eoff[b + 1]) ++k;
    bool all_owned = true;  // a vertex no element uses would belong to no patch
    for (int64_t v = voff[b]; v < voff[b + 1] && all_owned; ++v) all_owned = owned[v] != 0;
    (*eligible)[b] = eoff[b + 1] > eoff[b] && k - (*body_patch_off)[b] <= n_blocks && all_owned;
  }
  (*body_patch_off)[n_bodies] = k;
  return ISB_OK;
}

isb_status wave_order(int dim, int64_t n_v, int n_bodies, const int64_t* eoff, const int32_t* T, int64_t* perm) {
  constexpr int kWave = 64;
  const int nk = dim + 1;
  Patches pt;
  const isb_status st = build_patches(dim, n_v, n_bodies, eoff, T, kPatchMaxElems, patch_max_verts(dim), &pt);
  if (st != ISB_OK) return st;
  // bit w of mask[v * nk + k]: a wavefront group w of the current patch has vertex v in slot k
  std::vector<uint32_t> mask((size_t)n_v * nk, 0);
  std::vector<int> fill, cap;
  std::vector<int64_t> slots;
  const int64_t n_e = eoff[n_bodies];
  static_assert(kPatchMaxElems / kWave <= 32, "groups of one patch must fit the 32-bit mask");
  for (size_t q = 0; q + 1 < pt.eoff.size(); ++q) {
    const int64_t s = pt.eoff[q], e1 = pt.eoff[q + 1];
    const int len = (int)(e1 - s), nw = (len + kWave - 1) / kWave;
    fill.assign(nw, 0);
    cap.assign(nw, kWave);
    cap[nw - 1] = len - (nw - 1) * kWave;  // groups full but the last, as the kernel's lanes take them
    slots.assign((size_t)nw * kWave, 0);
    for (int64_t e = s; e < e1; ++e)
      for (int k = 0; k < nk; ++k) mask[(size_t)T[e * nk + k] * nk + k] = 0;
    int start = 0;
    for (int64_t e = s; e < e1; ++e) {
      const int32_t* t = T + e * nk;
      uint32_t used = 0;
      for (int k = 0; k < nk; ++k) used |= mask[(size_t)t[k] * nk + k];
      // the first group from a rotating start with room and no clash; else the fewest clashes
      int pick = -1;
      for (int j = 0; j < nw && pick < 0; ++j) {
        const int w = (start + j) % nw;
        if (fill[w] < cap[w] && !((used >> w) & 1u)) pick = w;
      }
      if (pick < 0) {
        int best = nk + 1;
        for (int w = 0; w < nw; ++w) {
          if (fill[w] >= cap[w]) continue;
          int c = 0;
          for (int k = 0; k < nk; ++k) c += (mask[(size_t)t[k] * nk + k] >> w) & 1u;
          if (c < best) {
            best = c;
            pick = w;
          }
        }
      }
      for (int k = 0; k < nk; ++k) mask[(size_t)t[k] * nk + k] |= 1u << pick;
      slots[(size_t)pick * kWave + fill[pick]++] = e;
      start = (pick + 1) % nw;
    }
    int64_t o = s;
    for (int w = 0; w < nw; ++w)
      for (int i = 0; i < fill[w]; ++i) perm[o++] = slots[(size_t)w * kWave + i];
  }
  // bank balance of each packed patch: the plan numbers a patch's vertices by sorted global id, and
  // the same patch comes back when the caller applies the order (a permutation inside the patch
  // takes the same vertex set, so the builder cuts where it cut before). Patches are independent:
  // threads take them from a shared counter, and each patch's result does not depend on which
  // thread took it or on how many started (the calling thread alone finishes the work if none can).
  const int n_patch = (int)pt.eoff.size() - 1;
  const int n_thr = std::max(1, std::min<int>({(int)std::thread::hardware_concurrency(), 16, n_patch}));
  std::atomic<int> next{0};
  auto balance_some = [&]() {
    std::vector<int32_t> tloc, order, newid;
    std::vector<int64_t> packed;
    for (int q = next++; q < n_patch; q = next++) {
      const int64_t s = pt.eoff[q];
      const int len = (int)(pt.eoff[q + 1] - s), nv = pt.voff[q + 1] - pt.voff[q];
      tloc.resize((size_t)len * nk);
      for (int i = 0; i < len; ++i)
        for (int k = 0; k < nk; ++k) tloc[(size_t)i * nk + k] = pt.lconn[(size_t)k * n_e + perm[s + i]];
      balance_patch(dim, len, nv, tloc.data(), true, nv, &order, &newid, false);
      packed.assign(perm + s, perm + s + len);
      for (int i = 0; i < len; ++i) perm[s + i] = packed[order[i]];
    }
  };
  std::vector<std::thread> pool;
  pool.reserve(n_thr);
  try {
    for (int t = 1; t < n_thr; ++t) pool.emplace_back(balance_some);
  } catch (const std::system_error&) {
    // fewer helper threads than asked for: the ones that started and this thread share the rest
  }
  balance_some();
  for (std::thread& th : pool) th.join();
  return ISB_OK;
}

}  // namespace isb

extern "C" {

const char* isb_last_error(void) { return isb::last_error(); }

const char* isb_version(void) { return "isb 0.1 (gfx950)"; }

isb_status isb_validate_mesh(int dim, int64_t n_v, const double* X, int64_t n_e, const int32_t* T,
                             int32_t n_bodies, const int64_t* body_v_off, const int64_t* body_e_off) {
  isb::clear_error();
  return isb::validate_mesh(dim, n_v, X, n_e, T, n_bodies, body_v_off, body_e_off);
}

isb_status isb_locality_order(int dim, int64_t n_v, const double* X, int64_t n_e, const int32_t* T,
                              int32_t n_bodies, const int64_t* body_e_off, int64_t* perm_out) {
  isb::clear_error();
  if ((dim != 2 && dim != 3) || n_v <= 0 || n_e < 0 || !X || (n_e > 0 && !T) || !perm_out || n_bodies < 0)
    return isb::fail(ISB_E_ARG, "isb_locality_order: bad argument");
  std::vector<int64_t> eoff{0, n_e};
  if (body_e_off) {
    eoff.assign(body_e_off, body_e_off + n_bodies + 1);
    if (eoff.front() != 0 || eoff.back() != n_e) return isb::fail(ISB_E_ARG, "isb_locality_order: bad body_e_off");
    for (int32_t b = 0; b < n_bodies; ++b)
      if (eoff[b + 1] < eoff[b]) return isb::fail(ISB_E_ARG, "isb_locality_order: bad body_e_off");
  }
  const int nk = dim + 1;
  // bounding box of the rest positions
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < n_v; ++v)
    for (int c = 0; c < dim; ++c) {
      lo[c] = std::min(lo[c], X[v * dim + c]);
      hi[c] = std::max(hi[c], X[v * dim + c]);
    }
  // Morton key of each element's rest centroid on one cubic lattice over the bounding box (one
  // scale for every axis, so that the key's cells stay cubic on elongated meshes): 21 bits per
  // axis in 3D, 31 in 2D, bits interleaved
  const int bits = dim == 3 ? 21 : 31;
  double span = 0.0;
  for (int c = 0; c < dim; ++c) span = std::max(span, hi[c] - lo[c]);
  if (!(span > 0.0)) span = 1.0;
  std::vector<uint64_t> key((size_t)n_e);
  for (int64_t e = 0; e < n_e; ++e) {
    uint64_t q[3] = {0, 0, 0};
    for (int c = 0; c < dim; ++c) {
      double m = 0.0;
      for (int k = 0; k < nk; ++k) {
        const int32_t v = T[e * nk + k];
        if (v < 0 || v >= n_v) return isb::fail(ISB_E_MESH, "isb_locality_order: vertex index out of range");
        m += X[(int64_t)v * dim + c];
      }
      m /= nk;
      double t = (m - lo[c]) / span;
      t = std::min(std::max(t, 0.0), 1.0);
      q[c] = (uint64_t)(t * (double)((1ull << bits) - 1));
    }
    uint64_t k = 0;
    for (int bit = bits - 1; bit >= 0; --bit)
      for (int c = dim - 1; c >= 0; --c) k = (k << 1) | ((q[c] >> bit) & 1ull);
    key[e] = k;
  }
  for (int64_t e = 0; e < n_e; ++e) perm_out[e] = e;
  for (size_t b = 0; b + 1 < eoff.size(); ++b)
    std::stable_sort(perm_out + eoff[b], perm_out + eoff[b + 1],
                     [&](int64_t a, int64_t c) { return key[a] < key[c]; });
  return ISB_OK;
}

isb_status isb_wave_order(int dim, int64_t n_v, int64_t n_e, const int32_t* T, int32_t n_bodies,
                          const int64_t* body_e_off, int64_t* perm_out) {
  isb::clear_error();
  if ((dim != 2 && dim != 3) || n_v <= 0 || n_e < 0 || (n_e > 0 && !T) || !perm_out || n_bodies < 0 ||
      (body_e_off && n_bodies < 1))
    return isb::fail(ISB_E_ARG, "isb_wave_order: bad argument");
  std::vector<int64_t> eoff{0, n_e};
  int32_t nb = 1;
  if (body_e_off) {
    eoff.assign(body_e_off, body_e_off + n_bodies + 1);
    nb = n_bodies;
    if (eoff.front() != 0 || eoff.back() != n_e) return isb::fail(ISB_E_ARG, "isb_wave_order: bad body_e_off");
    for (int32_t b = 0; b < n_bodies; ++b)
      if (eoff[b + 1] < eoff[b]) return isb::fail(ISB_E_ARG, "isb_wave_order: bad body_e_off");
  }
  for (int64_t i = 0; i < n_e * (dim + 1); ++i)
    if (T[i] < 0 || T[i] >= n_v) return isb::fail(ISB_E_MESH, "isb_wave_order: vertex index out of range");
  if (n_e == 0) return ISB_OK;
  return isb::wave_order(dim, n_v, nb, eoff.data(), T, perm_out);
}

isb_status isb_colour_elements(int dim, int64_t n_v, int64_t n_e, const int32_t* T, int32_t* colour_out,
                               int32_t* n_colours_out) {
  isb::clear_error();
  if ((dim != 2 && dim != 3) || n_v <= 0 || n_e <= 0 || !T || !colour_out || !n_colours_out)
    return isb::fail(ISB_E_ARG, "isb_colour_elements: bad argument");
  return isb::colour_elements(dim, n_v, n_e, T, colour_out, n_colours_out);
}

}  // extern "C"
