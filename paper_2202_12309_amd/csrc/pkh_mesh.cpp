// pkh_mesh.cpp -- host runtime behind the C-ABI of include/pkhydro.h.
//
// Owns the leaf list (Parthenon Sec. 2.1: same-size blocks, leaves of an
// oct-tree, Morton order), validates tilings and 2:1 balance, builds the
// device tables the kernels read (leaf info, per-level location maps,
// fine-coarse face records), manages device memory through the caller's
// callbacks, and enqueues the per-cycle kernel sequence on the handle's
// stream. No host synchronisation happens inside pkh_step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pkhydro.h"
#include "pkh_internal.h"

// Row pitch of the state arrays, in doubles: each padded row is rounded up
// to a multiple of PKH_ROW_ALIGN and the arrays start PKH_ROW_ALIGN - NG
// doubles into their allocation, so that the active cells of every row
// begin on a 128-byte line (1: no padding).
#ifndef PKH_ROW_ALIGN
#define PKH_ROW_ALIGN 16
#endif

using namespace pkh;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(PKH_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));            \
  } while (0)

constexpr int MAXL = 7;
static_assert(BC_PERIODIC == PKH_BC_PERIODIC && BC_OUTFLOW == PKH_BC_OUTFLOW && BC_REFLECT == PKH_BC_REFLECT,
              "device boundary kinds follow pkh_config.bc");

int64_t wrapl(int64_t a, int64_t n) {
  a %= n;
  return a < 0 ? a + n : a;
}

uint64_t spread_bits(uint64_t x) {
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((x >> b) & 1ull) << (3 * b);
  return r;
}

// ---------------------------------------------------------------------------
// Leaf set with per-level dense location maps.
// ---------------------------------------------------------------------------
struct Tree {
  int32_t nrb[3] = {1, 1, 1};
  int32_t maxl = 0;
  bool periodic[3] = {true, true, true};
  std::vector<pkh_loc> leaves;
  std::vector<std::vector<int32_t>> map;  // per level

  int64_t nbd(int L, int d) const { return (int64_t)nrb[d] << L; }

  // Block location (x,y,z) of level L wrapped along periodic directions;
  // false when it lies beyond a non-periodic face of the domain.
  bool inside(int L, int64_t& x, int64_t& y, int64_t& z) const {
    int64_t* c[3] = {&x, &y, &z};
    for (int d = 0; d < 3; ++d) {
      if (periodic[d])
        *c[d] = wrapl(*c[d], nbd(L, d));
      else if (*c[d] < 0 || *c[d] >= nbd(L, d))
        return false;
    }
    return true;
  }

  int32_t at(int L, int64_t x, int64_t y, int64_t z) const {
    if (L < 0 || L > maxl || !inside(L, x, y, z)) return -1;
    return map[L][(z * nbd(L, 1) + y) * nbd(L, 0) + x];
  }
  // Leaf at a coarser level containing block (x,y,z) of level L.
  int32_t coarser(int L, int64_t x, int64_t y, int64_t z, int* lc) const {
    if (!inside(L, x, y, z)) return -1;
    for (int c = L - 1; c >= 0; --c) {
      int s = L - c;
      int32_t id = at(c, x >> s, y >> s, z >> s);
      if (id >= 0) {
        *lc = c;
        return id;
      }
    }
    return -1;
  }

  uint64_t key(const pkh_loc& l) const {
    int s = maxl - l.level;
    return spread_bits((uint64_t)l.lx1 << s) | (spread_bits((uint64_t)l.lx2 << s) << 1) |
           (spread_bits((uint64_t)l.lx3 << s) << 2);
  }

  void sort_morton() {
    std::stable_sort(leaves.begin(), leaves.end(), [&](const pkh_loc& a, const pkh_loc& b) {
      uint64_t ka = key(a), kb = key(b);
      return ka != kb ? ka < kb : a.level < b.level;
    });
  }

  // Build the maps; check exact tiling and 2:1 balance over all 26
  // neighbour directions.
  int build() {
    map.assign(maxl + 1, {});
    for (int L = 0; L <= maxl; ++L) map[L].assign(nbd(L, 0) * nbd(L, 1) * nbd(L, 2), -1);
    const int64_t f0 = nbd(maxl, 0), f1 = nbd(maxl, 1), f2 = nbd(maxl, 2);
    std::vector<uint8_t> occ(f0 * f1 * f2, 0);
    for (size_t b = 0; b < leaves.size(); ++b) {
      const pkh_loc& l = leaves[b];
      if (l.level < 0 || l.level > maxl)
        return fail(PKH_EINVAL, "leaf %zu: level %d outside [0, %d]", b, l.level, maxl);
      const int64_t c[3] = {l.lx1, l.lx2, l.lx3};
      for (int d = 0; d < 3; ++d)
        if (c[d] < 0 || c[d] >= nbd(l.level, d))
          return fail(PKH_EINVAL, "leaf %zu: location out of range", b);
      map[l.level][(c[2] * nbd(l.level, 1) + c[1]) * nbd(l.level, 0) + c[0]] = (int32_t)b;
      const int s = maxl - l.level;
      for (int64_t z = c[2] << s; z < (c[2] + 1) << s; ++z)
        for (int64_t y = c[1] << s; y < (c[1] + 1) << s; ++y)
          for (int64_t x = c[0] << s; x < (c[0] + 1) << s; ++x) {
            uint8_t& o = occ[(z * f1 + y) * f0 + x];
            if (o) return fail(PKH_ETILING, "leaf %zu overlaps another leaf", b);
            o = 1;
          }
    }
    for (uint8_t o : occ)
      if (!o) return fail(PKH_ETILING, "the leaves leave part of the domain uncovered");
    for (size_t b = 0; b < leaves.size(); ++b) {
      const pkh_loc& l = leaves[b];
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            if (!dx && !dy && !dz) continue;
            int64_t x = l.lx1 + dx, y = l.lx2 + dy, z = l.lx3 + dz;
            if (!inside(l.level, x, y, z)) continue;  // beyond a wall: no neighbour
            if (at(l.level, x, y, z) >= 0) continue;
            int lc;
            if (coarser(l.level, x, y, z, &lc) >= 0) {
              if (lc < l.level - 1) return fail(PKH_EBALANCE, "leaf %zu: coarser neighbour two levels up", b);
              continue;
            }
            const int del[3] = {dx, dy, dz};
            for (int ch = 0; ch < 8; ++ch) {
              const int o[3] = {ch & 1, (ch >> 1) & 1, (ch >> 2) & 1};
              bool touch = true;
              for (int e = 0; e < 3; ++e)
                if ((del[e] < 0 && o[e] == 0) || (del[e] > 0 && o[e] == 1)) touch = false;
              if (!touch) continue;
              if (at(l.level + 1, 2 * x + o[0], 2 * y + o[1], 2 * z + o[2]) < 0)
                return fail(PKH_EBALANCE, "leaf %zu: finer neighbour two levels down", b);
            }
          }
    }
    return PKH_OK;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// The mesh handle.
// ---------------------------------------------------------------------------
struct pkh_mesh {
  pkh_config cfg{};
  hipStream_t stream = nullptr;
  int device = 0;  // the HIP device current at creation
  pkh_alloc_fn af = nullptr;
  pkh_free_fn ffn = nullptr;
  void* actx = nullptr;
  Tree tree;
  Geom g{};
  // device arrays
  double* A = nullptr;  // U^n / U^{n+1} with ghosts
  double* B = nullptr;  // U* with ghosts
  BlockInfo* d_blocks = nullptr;
  int32_t* d_map = nullptr;
  LevelMaps maps{};
  DevTime* d_time = nullptr;
  double* d_fbuf = nullptr;
  FineFace* d_ff = nullptr;
  int32_t* d_ff_first = nullptr;
  int32_t* d_cblocks = nullptr;
  int32_t ncblocks = 0;
  int32_t* d_nbr = nullptr;   // [leaf][27] same-level neighbours (-1: other level)
  bool need_fill = false;     // some ghost region has a neighbour at another level
  int32_t* d_jf = nullptr;    // (leaf, face) pairs whose face neighbour is on another level
  uint2* d_plan = nullptr;    // where each ghost-face thread reads (launch_fill_plan)
  int32_t njf = 0;
  // virtual partition into contiguous leaf ranges: same-level faces between
  // parts go through pack / transfer / unpack instead of direct reads
  int32_t nparts = 1;
  RemoteFace* d_rf = nullptr;
  int32_t nrf = 0;
  double* d_send = nullptr;
  double* d_recv = nullptr;
  int64_t rf_slot = 0;                            // doubles per remote face
  std::vector<std::array<int64_t, 2>> msgs;       // per (sender part, receiver part): first record, count
  double* d_partial = nullptr;
  double* d_tot = nullptr;
  size_t partial_cap = 0;
  std::vector<BlockInfo> h_blocks;
  std::vector<int8_t> flags;
  bool ghosts_valid = false;
  int32_t tj = 0;
  int32_t packs = 1;  // stage launches per stage (contiguous leaf ranges)
  // tapes and batches holding pointers into the leaf layout (regrid and
  // partition changes are refused while any is attached)
  int32_t attached = 0;
  // kernel timing: event pairs around launches of the selected kinds
  uint32_t kt_mask = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::array<int64_t, 3>> kt_rec;  // kind, start event, end event
  // captured cycles
  hipGraphExec_t gexec = nullptr;
  int32_t g_cycles = 0;
  double g_tend = NAN;
  bool g_valid = false;

  int64_t nb() const { return (int64_t)tree.leaves.size(); }
  bool fp32 = false;  // state stored in FP32 (single-level periodic meshes)
  size_t state_bytes() const { return (size_t)nb() * g.bstride * (fp32 ? sizeof(float) : sizeof(double)); }
  // A and B start this many doubles into their allocations (the row
  // alignment of the active cells)
  static constexpr int64_t state_head() { return (PKH_ROW_ALIGN - NG % PKH_ROW_ALIGN) % PKH_ROW_ALIGN; }
  // arrays in the padded block layout (states, the tape's recomputed
  // states and adjoint arrays), line-aligned like A and B
  double* padded_alloc(size_t bytes) {
    double* raw = (double*)dalloc(bytes + state_head() * sizeof(double));
    return raw ? raw + state_head() : nullptr;
  }
  void padded_free(double* p) {
    if (p) dfree(p - state_head());
  }
  double* state_alloc() { return padded_alloc(state_bytes()); }
  void state_free(double* p) { padded_free(p); }
  float* Af() const { return reinterpret_cast<float*>(A); }

  void* dalloc(size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (af) return af(bytes, stream, actx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
  }
  void dfree(void* p) {
    if (!p) return;
    if (ffn)
      ffn(p, stream, actx);
    else
      (void)hipFree(p);
  }
};

namespace {

void drop_graph(pkh_mesh* m) {
  if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
  m->gexec = nullptr;
  m->g_valid = false;
}

// The tables one cycle uses besides the block list and level maps (rebuilt
// on every regrid and partition change).
void free_cycle_tables(pkh_mesh* m) {
  m->dfree(m->d_fbuf);
  m->dfree(m->d_ff);
  m->dfree(m->d_ff_first);
  m->dfree(m->d_cblocks);
  m->dfree(m->d_jf);
  m->dfree(m->d_plan);
  m->dfree(m->d_nbr);
  m->dfree(m->d_rf);
  m->dfree(m->d_send);
  m->dfree(m->d_recv);
  m->d_fbuf = nullptr;
  m->d_ff = nullptr;
  m->d_ff_first = nullptr;
  m->d_cblocks = nullptr;
  m->d_jf = nullptr;
  m->d_plan = nullptr;
  m->d_nbr = nullptr;
  m->d_rf = nullptr;
  m->d_send = nullptr;
  m->d_recv = nullptr;
  m->njf = 0;
  m->ncblocks = 0;
  m->nrf = 0;
  m->msgs.clear();
}

void free_tables(pkh_mesh* m) {
  m->dfree(m->d_blocks);
  m->dfree(m->d_map);
  m->d_blocks = nullptr;
  m->d_map = nullptr;
  free_cycle_tables(m);
}

template <class T>
int upload_vec(pkh_mesh* m, T** dptr, const std::vector<T>& h) {
  *dptr = (T*)m->dalloc(std::max<size_t>(h.size(), 1) * sizeof(T));
  if (!*dptr) return fail(PKH_ENOMEM, "device allocation of %zu bytes failed", h.size() * sizeof(T));
  if (!h.empty())
    HIPCHK(hipMemcpyAsync(*dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, m->stream));
  return PKH_OK;
}

// Build BlockInfo, level maps and fine-coarse face records for the current
// leaf list, and upload them. The tree maps must be built.
int build_tables(pkh_mesh* m, std::vector<BlockInfo>& hb, int32_t** dmap, LevelMaps& lm) {
  const Tree& t = m->tree;
  const int64_t nb = m->nb();
  hb.assign(nb, BlockInfo{});
  for (int64_t b = 0; b < nb; ++b) {
    const pkh_loc& l = t.leaves[b];
    BlockInfo& bi = hb[b];
    bi.level = l.level;
    bi.lx = l.lx1;
    bi.ly = l.lx2;
    bi.lz = l.lx3;
    for (int d = 0; d < 3; ++d) {
      const double ncell = (double)((int64_t)m->cfg.nroot[d] << l.level);
      bi.idx[d] = ncell / (m->cfg.xmax[d] - m->cfg.xmin[d]);
    }
    for (int f = 0; f < 6; ++f) bi.fslot[f] = -1;
    bi.finer_mask = 0;
  }
  // fine-coarse faces: a coarse leaf's face borders finer leaves when the
  // same-level neighbour location is neither a leaf nor inside a coarser one
  std::vector<FineFace> ff;
  std::vector<int32_t> ff_first, cblocks;
  int32_t nslot = 0;
  std::vector<std::array<int32_t, 6>> slot_of(nb);
  for (auto& s : slot_of) s.fill(-1);
  auto slot = [&](int64_t b, int f) {
    if (slot_of[b][f] < 0) slot_of[b][f] = nslot++;
    return slot_of[b][f];
  };
  for (int64_t b = 0; b < nb; ++b) {
    const pkh_loc& l = t.leaves[b];
    bool any = false;
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1, s = f & 1;
      int64_t c[3] = {l.lx1, l.lx2, l.lx3};
      c[d] += s ? 1 : -1;
      if (!t.inside(l.level, c[0], c[1], c[2])) continue;  // domain boundary
      if (t.at(l.level, c[0], c[1], c[2]) >= 0) continue;
      int lc;
      if (t.coarser(l.level, c[0], c[1], c[2], &lc) >= 0) continue;
      // finer: the 4 children of c touching this face
      FineFace rec{};
      rec.block = (int32_t)b;
      rec.face = f;
      rec.own_slot = slot(b, f);
      const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      for (int h2 = 0; h2 < 2; ++h2)
        for (int h1 = 0; h1 < 2; ++h1) {
          int64_t ch[3];
          ch[d] = 2 * c[d] + (s ? 0 : 1);
          ch[t1] = 2 * c[t1] + h1;
          ch[t2] = 2 * c[t2] + h2;
          const int32_t fid = t.at(l.level + 1, ch[0], ch[1], ch[2]);
          if (fid < 0) return fail(PKH_EBALANCE, "fine face without fine leaves");
          rec.fine_slot[h1 + 2 * h2] = slot(fid, f ^ 1);
        }
      if (!any) {
        ff_first.push_back((int32_t)ff.size());
        cblocks.push_back((int32_t)b);
        any = true;
      }
      hb[b].finer_mask |= 1 << f;
      ff.push_back(rec);
    }
  }
  ff_first.push_back((int32_t)ff.size());
  for (int64_t b = 0; b < nb; ++b)
    for (int f = 0; f < 6; ++f) hb[b].fslot[f] = slot_of[b][f];
  // same-level neighbour table
  std::vector<int32_t> nbr(nb * 27, -1);
  bool need_fill = false;
  for (int64_t b = 0; b < nb; ++b) {
    const pkh_loc& l = t.leaves[b];
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dx && !dy && !dz) continue;
          const int32_t id = t.at(l.level, l.lx1 + dx, l.lx2 + dy, l.lx3 + dz);
          nbr[b * 27 + (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] = id;
          if (id < 0) need_fill = true;
        }
  }
  // faces whose neighbour is on another level or beyond a wall: the ghost
  // regions the stage kernels read from the ghost zone (all same-level halos
  // are read from the neighbours' active cells). Record: leaf, then face
  // | boundary kind << 3 (kind 0: a level jump).
  std::vector<int32_t> jf;
  for (int64_t b = 0; b < nb; ++b) {
    static const int slot[6] = {12, 14, 10, 16, 4, 22};
    const pkh_loc& l = t.leaves[b];
    for (int f = 0; f < 6; ++f)
      if (nbr[b * 27 + slot[f]] < 0) {
        int64_t c[3] = {l.lx1, l.lx2, l.lx3};
        c[f >> 1] += (f & 1) ? 1 : -1;
        const int kind = t.inside(l.level, c[0], c[1], c[2]) ? 0 : m->cfg.bc[f];
        // a level jump to a coarser leaf (2:1 balance: one level up), else
        // a refined face (t.inside above wrapped c along periodic axes)
        const int coarser = kind == 0 && l.level > 0 && t.at(l.level - 1, c[0] >> 1, c[1] >> 1, c[2] >> 1) >= 0;
        jf.push_back((int32_t)b);
        jf.push_back(f | kind << 3 | coarser << 6);
      }
  }
  // remote faces of a partitioned mesh: a same-level face neighbour in another
  // part is read from the ghost zone, which pack / transfer / unpack fill
  std::vector<RemoteFace> rf;
  std::vector<std::array<int64_t, 2>> msgs;
  const int32_t P = dmap == &m->d_map ? std::max(1, std::min<int32_t>(m->nparts, (int32_t)nb)) : 1;
  if (P > 1) {
    std::vector<int32_t> part_of(nb);  // part p holds leaves [p nb / P, (p+1) nb / P)
    for (int32_t p = 0; p < P; ++p)
      for (int64_t b = (int64_t)p * nb / P; b < (int64_t)(p + 1) * nb / P; ++b) part_of[b] = p;
    auto part = [&](int64_t b) { return part_of[b]; };
    std::vector<std::vector<RemoteFace>> by_pair((size_t)P * P);
    static const int slot[6] = {12, 14, 10, 16, 4, 22};
    for (int64_t b = 0; b < nb; ++b)
      for (int f = 0; f < 6; ++f) {
        const int32_t s = nbr[b * 27 + slot[f]];
        if (s >= 0 && part(s) != part(b)) by_pair[(size_t)part(s) * P + part(b)].push_back({(int32_t)b, f, s, 0});
      }
    for (const auto& v : by_pair) {
      if (v.empty()) continue;
      msgs.push_back({(int64_t)rf.size(), (int64_t)v.size()});
      rf.insert(rf.end(), v.begin(), v.end());
    }
    for (const RemoteFace& r : rf) nbr[(int64_t)r.recv * 27 + slot[r.face]] = -1;
    if (!rf.empty()) need_fill = true;
  }
  // level maps
  std::vector<int32_t> flat;
  for (int L = 0; L <= t.maxl; ++L) {
    lm.off[L] = (int64_t)flat.size();
    for (int d = 0; d < 3; ++d) lm.nb[L][d] = (int32_t)t.nbd(L, d);
    flat.insert(flat.end(), t.map[L].begin(), t.map[L].end());
  }
  lm.maxl = t.maxl;
  int rc;
  if ((rc = upload_vec(m, dmap, flat))) return rc;
  lm.map = *dmap;
  // per-mesh AMR tables (only the current mesh's are kept)
  if (dmap == &m->d_map) {
    if ((rc = upload_vec(m, &m->d_blocks, hb))) return rc;
    const size_t fsz = (size_t)NV *
                       std::max({m->g.n1 * m->g.n2, m->g.n1 * m->g.n3, m->g.n2 * m->g.n3});
    m->d_fbuf = (double*)m->dalloc(std::max<size_t>(nslot, 1) * fsz * sizeof(double));
    if (!m->d_fbuf) return fail(PKH_ENOMEM, "face buffer allocation failed");
    if ((rc = upload_vec(m, &m->d_ff, ff))) return rc;
    if ((rc = upload_vec(m, &m->d_ff_first, ff_first))) return rc;
    if ((rc = upload_vec(m, &m->d_cblocks, cblocks))) return rc;
    m->ncblocks = (int32_t)cblocks.size();
    if ((rc = upload_vec(m, &m->d_nbr, nbr))) return rc;
    m->need_fill = need_fill;
    m->njf = (int32_t)(jf.size() / 2);
    if (m->njf && (rc = upload_vec(m, &m->d_jf, jf))) return rc;
    if (m->njf) {
      m->d_plan = (uint2*)m->dalloc((size_t)m->njf * fill_faces_stride(m->g) * sizeof(uint2));
      if (!m->d_plan) return fail(PKH_ENOMEM, "face-fill plan allocation failed");
      HIPCHK(launch_fill_plan(m->d_plan, m->d_blocks, m->g, lm, m->d_jf, m->njf, m->stream));
    }
    m->nrf = (int32_t)rf.size();
    m->msgs = msgs;
    m->rf_slot = 2 * (int64_t)NV * std::max({m->g.n1 * m->g.n2, m->g.n1 * m->g.n3, m->g.n2 * m->g.n3});
    if (m->nrf) {
      if ((rc = upload_vec(m, &m->d_rf, rf))) return rc;
      const size_t bytes = (size_t)m->nrf * m->rf_slot * sizeof(double);
      m->d_send = (double*)m->dalloc(bytes);
      m->d_recv = (double*)m->dalloc(bytes);
      if (!m->d_send || !m->d_recv) return fail(PKH_ENOMEM, "remote-face buffer allocation failed");
    }
  }
  // the host vectors above are sources of asynchronous copies
  HIPCHK(hipStreamSynchronize(m->stream));
  return PKH_OK;
}

int ensure_partials(pkh_mesh* m) {
  const size_t need = (size_t)m->nb() * NV;
  if (m->partial_cap >= need && m->d_partial) return PKH_OK;
  m->dfree(m->d_partial);
  m->d_partial = (double*)m->dalloc(need * sizeof(double));
  if (!m->d_partial) return fail(PKH_ENOMEM, "partial-sum allocation failed");
  m->partial_cap = need;
  return PKH_OK;
}

int check_err(pkh_mesh* m) {
  DevTime h;
  HIPCHK(hipMemcpyAsync(&h, m->d_time, sizeof h, hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  if (h.err & 4)
    return fail(PKH_ESTATE, "a bounded wait of a persistent batch launch gave up: the state is invalid");
  if (h.err & 2) return fail(PKH_EBALANCE, "a ghost or regrid lookup found no covering leaf");
  if (h.err & 1) return fail(PKH_EPHYS, "unphysical state (rho <= 0, P <= 0 or non-finite)");
  return PKH_OK;
}

// The CFL timestep of the current state (dt_kernel, then the clock).
int refresh_dt(pkh_mesh* m) {
  HIPCHK(hipMemsetAsync(&m->d_time->smax_bits, 0, sizeof(unsigned long long), m->stream));
  if (m->fp32)
    HIPCHK(launch_dt(m->Af(), m->d_blocks, (int32_t)m->nb(), m->g, m->d_time, m->stream));
  else
    HIPCHK(launch_dt(m->A, m->d_blocks, (int32_t)m->nb(), m->g, m->d_time, m->stream));
  HIPCHK(launch_clock(m->d_time, CLOCK_FROM_SMAX, NAN, m->stream));
  return PKH_OK;
}

int do_exchange(pkh_mesh* m) {
  // an FP32-stored mesh is single-level and periodic: the stage kernels read
  // every halo cell from a neighbour, so no ghost zone is ever read
  if (!m->fp32)
    HIPCHK(launch_fill(m->A, m->d_blocks, (int32_t)m->nb(), m->g, m->maps, m->d_time, 0, m->stream));
  int rc;
  if ((rc = refresh_dt(m))) return rc;
  m->ghosts_valid = true;
  return PKH_OK;
}

hipEvent_t next_event(pkh_mesh* m) {
  if (m->ev_used == m->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    m->ev_pool.push_back(e);
  }
  return m->ev_pool[m->ev_used++];
}

// Bracket a launch of kind index k with events when timing is on and the
// stream is not being captured.
struct KTimer {
  pkh_mesh* m;
  int k;
  int64_t s = -1;
  bool on;
  KTimer(pkh_mesh* mm, int kind, bool capturing) : m(mm), k(kind) {
    on = !capturing && ((m->kt_mask >> k) & 1u);
    if (on) {
      hipEvent_t e = next_event(m);
      if (e && hipEventRecord(e, m->stream) == hipSuccess) s = (int64_t)(m->ev_used - 1);
    }
  }
  ~KTimer() {
    if (on && s >= 0) {
      hipEvent_t e = next_event(m);
      if (e && hipEventRecord(e, m->stream) == hipSuccess)
        m->kt_rec.push_back({k, s, (int64_t)(m->ev_used - 1)});
    }
  }
};

// Ghost layers of the remote faces of state u: pack, one transfer per
// (sender part, receiver part) message, unpack. On one GPU the transfer is a
// device copy; across GPUs it would be the peer send / receive.
int exchange_remote(pkh_mesh* m, double* u, bool capturing) {
  if (!m->nrf) return PKH_OK;
  KTimer kt(m, 5, capturing);
  HIPCHK(launch_remote_pack(u, m->d_rf, m->nrf, m->g, m->d_send, m->rf_slot, m->stream));
  for (const auto& msg : m->msgs)
    HIPCHK(hipMemcpyAsync(m->d_recv + msg[0] * m->rf_slot, m->d_send + msg[0] * m->rf_slot,
                          (size_t)msg[1] * m->rf_slot * sizeof(double), hipMemcpyDeviceToDevice, m->stream));
  HIPCHK(launch_remote_unpack(u, m->d_rf, m->nrf, m->g, m->d_recv, m->rf_slot, m->stream));
  return PKH_OK;
}

// One cycle's kernels (the clock BEGIN of the cycle has been enqueued).
int enqueue_cycle(pkh_mesh* m, int mode_after, double t_end, bool capturing = false) {
  int rc;
  const int32_t nb = (int32_t)m->nb();
  StageLaunch s{};
  s.blocks = m->d_blocks;
  s.nblocks = nb;
  s.g = m->g;
  s.tm = m->d_time;
  s.fbuf = m->d_fbuf;
  s.nbr = m->d_nbr;
  s.tj = m->tj;
  s.fp32 = m->fp32;
  // one launch per pack: leaves [p nb / P, (p+1) nb / P)
  const int32_t P = std::max(1, std::min(m->packs, nb));
  auto launch_packs = [&](StageLaunch st) -> hipError_t {
    for (int32_t p = 0; p < P; ++p) {
      st.b0 = (int32_t)((int64_t)p * nb / P);
      st.nblocks = (int32_t)((int64_t)(p + 1) * nb / P) - st.b0;
      const hipError_t e = launch_stage(st, m->stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  // predictor: U* = U^n - dt/2 D(U^n)
  s.uin = m->A;
  s.ubase = m->A;
  s.uout = m->B;
  s.beta = 0.5;
  s.recon = m->cfg.stage1_recon;
  s.do_dt = 0;
  {
    KTimer kt(m, 0, capturing);
    HIPCHK(launch_packs(s));
  }
  if (m->ncblocks) {
    KTimer kt(m, 3, capturing);
    HIPCHK(launch_flux_correct(m->B, m->d_blocks, m->d_ff, m->d_ff_first, m->d_cblocks,
                               m->ncblocks, m->g, m->d_time, 0.5, 0, m->d_fbuf, m->d_nbr,
                               m->stream));
  }
  if ((rc = exchange_remote(m, m->B, capturing))) return rc;
  if (m->njf) {  // ghost faces across level jumps (same-level halos are read directly)
    KTimer kt(m, 2, capturing);
    HIPCHK(launch_fill_faces(m->B, m->g, m->d_time, m->d_jf, m->d_plan, m->njf, m->stream));
  }
  // corrector: U^{n+1} = U^n - dt D_PLM(U*), in place; CFL reduction fused
  s.uin = m->B;
  s.ubase = m->A;
  s.uout = m->A;
  s.beta = 1.0;
  s.recon = PKH_RECON_PLM;
  s.do_dt = 1;
  {
    KTimer kt(m, 1, capturing);
    HIPCHK(launch_packs(s));
  }
  if (m->ncblocks) {
    KTimer kt(m, 3, capturing);
    HIPCHK(launch_flux_correct(m->A, m->d_blocks, m->d_ff, m->d_ff_first, m->d_cblocks,
                               m->ncblocks, m->g, m->d_time, 1.0, 1, m->d_fbuf, m->d_nbr,
                               m->stream));
  }
  if ((rc = exchange_remote(m, m->A, capturing))) return rc;
  if (m->njf) {
    KTimer kt(m, 2, capturing);
    HIPCHK(launch_fill_faces(m->A, m->g, m->d_time, m->d_jf, m->d_plan, m->njf, m->stream));
  }
  HIPCHK(launch_clock(m->d_time, mode_after, t_end, m->stream));
  return PKH_OK;
}

int check_config(const pkh_config* c) {
  if (c->nghost != 2) return fail(PKH_EINVAL, "nghost must be 2");
  if (c->max_level < 0 || c->max_level > MAXL) return fail(PKH_EINVAL, "max_level must be in [0, %d]", MAXL);
  const int n1 = c->nblock[0];
  if (n1 != 8 && n1 != 16 && n1 != 32 && n1 != 64)
    return fail(PKH_EINVAL, "nblock[0] must be 8, 16, 32 or 64 (got %d)", n1);
  const int tj = n1 == 64 ? 4 : 8;
  for (int d = 0; d < 3; ++d) {
    if (c->nblock[d] < 4 || c->nroot[d] % c->nblock[d])
      return fail(PKH_EINVAL, "nroot[%d]=%d must be a multiple of nblock[%d]=%d >= 4", d, c->nroot[d], d,
                  c->nblock[d]);
    if (c->max_level > 0 && (c->nblock[d] < 8 || (c->nblock[d] & 1)))
      return fail(PKH_EINVAL, "multilevel meshes need even nblock >= 8");
    if (!(c->xmax[d] > c->xmin[d])) return fail(PKH_EINVAL, "xmax must exceed xmin");
  }
  if (c->nblock[1] % tj) return fail(PKH_EINVAL, "nblock[1] must be a multiple of %d", tj);
  for (int f = 0; f < 6; ++f) {
    if (c->bc[f] != PKH_BC_PERIODIC && c->bc[f] != PKH_BC_OUTFLOW && c->bc[f] != PKH_BC_REFLECT)
      return fail(PKH_EINVAL, "bc[%d] = %d is not a boundary kind", f, c->bc[f]);
    if ((c->bc[f] == PKH_BC_PERIODIC) != (c->bc[f ^ 1] == PKH_BC_PERIODIC))
      return fail(PKH_EINVAL, "a periodic direction must be periodic on both faces");
  }
  if (c->flags & PKH_FLAG_FP32_STATE) {
    if (c->max_level != 0) return fail(PKH_EINVAL, "FP32 state storage needs max_level 0");
    for (int f = 0; f < 6; ++f)
      if (c->bc[f] != PKH_BC_PERIODIC) return fail(PKH_EINVAL, "FP32 state storage needs periodic boundaries");
    if (n1 != 16 && n1 != 32) return fail(PKH_EINVAL, "FP32 state storage needs nblock[0] of 16 or 32");
  }
  if (c->stage1_recon != PKH_RECON_DC && c->stage1_recon != PKH_RECON_PLM)
    return fail(PKH_EINVAL, "stage1_recon must be PKH_RECON_DC or PKH_RECON_PLM");
  if (c->limiter != PKH_LIMITER_MC) return fail(PKH_EINVAL, "only the MC limiter is supported");
  if (!(c->gamma > 1.0) || !(c->cfl > 0.0)) return fail(PKH_EINVAL, "need gamma > 1 and cfl > 0");
  return PKH_OK;
}

// clear: zero both arrays (at creation). A regrid skips it: the regrid
// kernel writes every active cell of A, the face fill its ghost faces, and
// the cycle writes B before reading it; no kernel reads the rest (the
// other ghost regions, the row padding).
int alloc_state(pkh_mesh* m, bool clear = true) {
  m->A = m->state_alloc();
  m->B = m->state_alloc();
  if (!m->A || !m->B) return fail(PKH_ENOMEM, "state allocation of 2 x %zu bytes failed", m->state_bytes());
  if (clear) {
    HIPCHK(hipMemsetAsync(m->A, 0, m->state_bytes(), m->stream));
    HIPCHK(hipMemsetAsync(m->B, 0, m->state_bytes(), m->stream));
  }
  return PKH_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* pkh_last_error(void) { return g_err.c_str(); }

int pkh_mesh_create(const pkh_config* cfg, const pkh_loc* blocks, int64_t nblocks, void* hip_stream,
                    pkh_alloc_fn alloc, pkh_free_fn free_fn, void* alloc_ctx, pkh_mesh** out) {
  g_err.clear();
  if (!cfg || !blocks || !out || nblocks <= 0) return fail(PKH_EINVAL, "null argument or no blocks");
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) return fail(PKH_EINVAL, "alloc and free go together");
  int rc = check_config(cfg);
  if (rc) return rc;
  pkh_mesh* m = new pkh_mesh();
  m->cfg = *cfg;
  m->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return fail(PKH_EHIP, "no current HIP device");
  }
  m->af = alloc;
  m->ffn = free_fn;
  m->actx = alloc_ctx;
  for (int d = 0; d < 3; ++d) {
    m->tree.nrb[d] = cfg->nroot[d] / cfg->nblock[d];
    m->tree.periodic[d] = cfg->bc[2 * d] == PKH_BC_PERIODIC;
  }
  m->tree.maxl = cfg->max_level;
  m->fp32 = (cfg->flags & PKH_FLAG_FP32_STATE) != 0;
  m->tree.leaves.assign(blocks, blocks + nblocks);
  m->tree.sort_morton();
  if ((rc = m->tree.build())) {
    delete m;
    return rc;
  }
  Geom& g = m->g;
  g.n1 = cfg->nblock[0];
  g.n2 = cfg->nblock[1];
  g.n3 = cfg->nblock[2];
  g.p1 = (g.n1 + 2 * NG + PKH_ROW_ALIGN - 1) / PKH_ROW_ALIGN * PKH_ROW_ALIGN;
  g.p2 = g.n2 + 2 * NG;
  g.p3 = g.n3 + 2 * NG;
  g.vstride = (int64_t)g.p1 * g.p2 * g.p3;
  g.bstride = NV * g.vstride;
  for (int d = 0; d < 3; ++d) g.nrb[d] = m->tree.nrb[d];
  for (int f = 0; f < 6; ++f) g.bc[f] = cfg->bc[f];
  g.gamma = cfg->gamma;
  m->d_time = (DevTime*)m->dalloc(sizeof(DevTime));
  if (!m->d_time) {
    delete m;
    return fail(PKH_ENOMEM, "allocation failed");
  }
  DevTime h{};
  h.cfl = cfg->cfl;
  if (hipMemcpyAsync(m->d_time, &h, sizeof h, hipMemcpyHostToDevice, m->stream) != hipSuccess ||
      (rc = alloc_state(m)) || (rc = build_tables(m, m->h_blocks, &m->d_map, m->maps)) ||
      (rc = ensure_partials(m))) {
    if (!rc) rc = fail(PKH_EHIP, "device setup failed");
    pkh_mesh_destroy(m);
    return rc;
  }
  m->d_tot = (double*)m->dalloc(NV * sizeof(double));
  if (!m->d_tot) {
    pkh_mesh_destroy(m);
    return fail(PKH_ENOMEM, "allocation failed");
  }
  m->flags.assign(m->nb(), 0);
  if (hipStreamSynchronize(m->stream) != hipSuccess) {
    pkh_mesh_destroy(m);
    return fail(PKH_EHIP, "stream synchronisation failed");
  }
  *out = m;
  return PKH_OK;
}

int pkh_mesh_destroy(pkh_mesh* m) {
  if (!m) return PKH_OK;
  (void)hipStreamSynchronize(m->stream);
  drop_graph(m);
  for (hipEvent_t e : m->ev_pool) (void)hipEventDestroy(e);
  free_tables(m);
  m->state_free(m->A);
  m->state_free(m->B);
  m->dfree(m->d_time);
  m->dfree(m->d_partial);
  m->dfree(m->d_tot);
  delete m;
  return PKH_OK;
}

int pkh_mesh_blocks(const pkh_mesh* m, pkh_loc* out, int64_t cap, int64_t* n) {
  if (!m || !n || (cap > 0 && !out)) return fail(PKH_EINVAL, "null argument");
  const int64_t nb = m->nb();
  *n = nb;
  std::copy(m->tree.leaves.begin(), m->tree.leaves.begin() + std::min(cap, nb), out);
  return PKH_OK;
}

int pkh_state_upload(pkh_mesh* m, const double* src, int32_t src_on_device) {
  if (!m || !src) return fail(PKH_EINVAL, "null argument");
  const size_t bytes = (size_t)m->nb() * NV * m->g.n1 * m->g.n2 * m->g.n3 * sizeof(double);
  const double* dsrc = src;
  double* stage = nullptr;
  if (!src_on_device) {
    stage = (double*)m->dalloc(bytes);
    if (!stage) return fail(PKH_ENOMEM, "staging allocation failed");
    HIPCHK(hipMemcpyAsync(stage, src, bytes, hipMemcpyHostToDevice, m->stream));
    dsrc = stage;
  }
  if (m->fp32)
    HIPCHK(launch_scatter(m->Af(), dsrc, (int32_t)m->nb(), m->g, m->stream));
  else
    HIPCHK(launch_scatter(m->A, dsrc, (int32_t)m->nb(), m->g, m->stream));
  HIPCHK(hipMemsetAsync(&m->d_time->err, 0, sizeof(int), m->stream));
  if (stage) {
    HIPCHK(hipStreamSynchronize(m->stream));
    m->dfree(stage);
  }
  m->ghosts_valid = false;
  return PKH_OK;
}

int pkh_state_download(pkh_mesh* m, double* dst, int32_t dst_on_device) {
  if (!m || !dst) return fail(PKH_EINVAL, "null argument");
  const size_t bytes = (size_t)m->nb() * NV * m->g.n1 * m->g.n2 * m->g.n3 * sizeof(double);
  double* ddst = dst;
  double* stage = nullptr;
  if (!dst_on_device) {
    stage = (double*)m->dalloc(bytes);
    if (!stage) return fail(PKH_ENOMEM, "staging allocation failed");
    ddst = stage;
  }
  if (m->fp32)
    HIPCHK(launch_gather(ddst, m->Af(), (int32_t)m->nb(), m->g, m->stream));
  else
    HIPCHK(launch_gather(ddst, m->A, (int32_t)m->nb(), m->g, m->stream));
  if (stage) HIPCHK(hipMemcpyAsync(dst, stage, bytes, hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  if (stage) m->dfree(stage);
  return check_err(m);
}

int pkh_exchange_boundaries(pkh_mesh* m) {
  if (!m) return fail(PKH_EINVAL, "null mesh");
  return do_exchange(m);
}

int pkh_step(pkh_mesh* m, int32_t n_cycles, double t_end) {
  if (!m || n_cycles < 0) return fail(PKH_EINVAL, "bad argument");
  if (n_cycles == 0) return PKH_OK;
  int rc;
  if (!m->ghosts_valid && (rc = do_exchange(m))) return rc;
  HIPCHK(launch_clock(m->d_time, CLOCK_BEGIN, t_end, m->stream));
  const bool graph = (m->cfg.flags & PKH_FLAG_GRAPH) != 0;
  if (!graph) {
    for (int c = 0; c < n_cycles; ++c)
      if ((rc = enqueue_cycle(m, c + 1 < n_cycles ? (CLOCK_END | CLOCK_BEGIN) : CLOCK_END, t_end)))
        return rc;
    return PKH_OK;
  }
  // Graph path: one captured cycle (ending with END|BEGIN) replayed; the
  // last cycle is enqueued eagerly so that it ends with END only.
  const bool same_tend = (std::isnan(t_end) && std::isnan(m->g_tend)) || t_end == m->g_tend;
  if (!m->g_valid || !same_tend) {
    drop_graph(m);
    hipGraph_t graph_h = nullptr;
    HIPCHK(hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal));
    rc = enqueue_cycle(m, CLOCK_END | CLOCK_BEGIN, t_end, true);
    hipError_t e = hipStreamEndCapture(m->stream, &graph_h);
    if (rc) return rc;
    if (e != hipSuccess) return fail(PKH_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&m->gexec, graph_h, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph_h);
    if (e != hipSuccess) return fail(PKH_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
    m->g_tend = t_end;
    m->g_valid = true;
  }
  for (int c = 0; c + 1 < n_cycles; ++c) HIPCHK(hipGraphLaunch(m->gexec, m->stream));
  return enqueue_cycle(m, CLOCK_END, t_end);
}

int pkh_get_time(pkh_mesh* m, double* t, double* dt, int64_t* cycle) {
  if (!m) return fail(PKH_EINVAL, "null mesh");
  if (!m->ghosts_valid) {
    int rc = do_exchange(m);
    if (rc) return rc;
  }
  DevTime h;
  HIPCHK(hipMemcpyAsync(&h, m->d_time, sizeof h, hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  if (t) *t = h.t;
  if (dt) *dt = h.dt_next;
  if (cycle) *cycle = h.cycle;
  if (h.err & 1) return fail(PKH_EPHYS, "unphysical state (rho <= 0, P <= 0 or non-finite)");
  if (h.err & 4)
    return fail(PKH_ESTATE, "a bounded wait of a persistent batch launch gave up: the state is invalid");
  if (h.err & 2) return fail(PKH_EBALANCE, "a ghost or regrid lookup found no covering leaf");
  return PKH_OK;
}

int pkh_set_time(pkh_mesh* m, double t, int64_t cycle) {
  if (!m) return fail(PKH_EINVAL, "null mesh");
  DevTime h;
  HIPCHK(hipMemcpyAsync(&h, m->d_time, sizeof h, hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  h.t = t;
  h.cycle = cycle;
  HIPCHK(hipMemcpyAsync(m->d_time, &h, sizeof h, hipMemcpyHostToDevice, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return PKH_OK;
}

int pkh_set_refinement_flags(pkh_mesh* m, const int8_t* flags, int64_t n) {
  if (!m || !flags || n != m->nb()) return fail(PKH_EINVAL, "need one flag per leaf");
  for (int64_t b = 0; b < n; ++b)
    if (flags[b] < -1 || flags[b] > 1) return fail(PKH_EINVAL, "flags must be -1, 0 or +1");
  m->flags.assign(flags, flags + n);
  return PKH_OK;
}

int pkh_flag_jump(pkh_mesh* m, int32_t quantity, double refine_above, double derefine_below, int8_t* flags_out,
                  double* eta_out) {
  if (!m) return fail(PKH_EINVAL, "null mesh");
  if (m->fp32) return fail(PKH_EINVAL, "refinement indicators need an FP64-stored state");
  if (quantity != PKH_JUMP_PRESSURE && quantity != PKH_JUMP_DENSITY)
    return fail(PKH_EINVAL, "quantity must be PKH_JUMP_PRESSURE or PKH_JUMP_DENSITY");
  if (!(derefine_below <= refine_above)) return fail(PKH_EINVAL, "derefine threshold above refine threshold");
  int rc;
  if (!m->ghosts_valid && (rc = do_exchange(m))) return rc;
  if ((rc = ensure_partials(m))) return rc;
  const int64_t nb = m->nb();
  std::vector<double> eta(nb);
  HIPCHK(launch_eta(m->d_partial, m->A, m->d_nbr, (int32_t)nb, m->g, quantity, m->stream));
  HIPCHK(hipMemcpyAsync(eta.data(), m->d_partial, nb * sizeof(double), hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  if ((rc = check_err(m))) return rc;
  m->flags.assign(nb, 0);
  for (int64_t b = 0; b < nb; ++b) {
    if (!(eta[b] == eta[b])) return fail(PKH_EPHYS, "non-finite jump indicator in leaf %lld", (long long)b);
    m->flags[b] = eta[b] > refine_above ? 1 : (eta[b] < derefine_below ? -1 : 0);
  }
  if (flags_out) std::copy(m->flags.begin(), m->flags.end(), flags_out);
  if (eta_out) std::copy(eta.begin(), eta.end(), eta_out);
  return PKH_OK;
}

int pkh_flag_pressure_jump(pkh_mesh* m, double refine_above, double derefine_below, int8_t* flags_out,
                           double* eta_out) {
  return pkh_flag_jump(m, PKH_JUMP_PRESSURE, refine_above, derefine_below, flags_out, eta_out);
}

int pkh_regrid(pkh_mesh* m) {
  if (!m) return fail(PKH_EINVAL, "null mesh");
  if (m->attached)
    return fail(PKH_ESTATE, "%d tape(s) or batch(es) hold this mesh's layout; destroy them before a regrid",
                m->attached);
  const Tree& t = m->tree;
  const int64_t nl = m->nb();
  std::vector<char> ref(nl, 0), der(nl, 0);
  for (int64_t b = 0; b < nl; ++b) ref[b] = m->flags[b] > 0 && t.leaves[b].level < t.maxl;
  // a refining leaf forces every touching coarser leaf to refine
  for (bool changed = true; changed;) {
    changed = false;
    for (int64_t b = 0; b < nl; ++b) {
      if (!ref[b]) continue;
      const pkh_loc& l = t.leaves[b];
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            if (!dx && !dy && !dz) continue;
            int lc;
            const int32_t c = t.coarser(l.level, l.lx1 + dx, l.lx2 + dy, l.lx3 + dz, &lc);
            if (c >= 0 && !ref[c]) {
              ref[c] = 1;
              changed = true;
            }
          }
    }
  }
  // merges: complete sibling groups all flagged -1, none refining, and the
  // parent keeps 2:1 with the refined mesh
  for (int64_t b = 0; b < nl; ++b) {
    const pkh_loc& l = t.leaves[b];
    if (l.level == 0 || (l.lx1 & 1) || (l.lx2 & 1) || (l.lx3 & 1)) continue;
    int32_t sib[8];
    bool ok = true;
    for (int c = 0; c < 8 && ok; ++c) {
      sib[c] = t.at(l.level, l.lx1 + (c & 1), l.lx2 + ((c >> 1) & 1), l.lx3 + ((c >> 2) & 1));
      if (sib[c] < 0 || m->flags[sib[c]] >= 0 || ref[sib[c]]) ok = false;
    }
    if (!ok) continue;
    const int L = l.level;
    const int64_t p[3] = {l.lx1 >> 1, l.lx2 >> 1, l.lx3 >> 1};
    for (int dz = -1; dz <= 1 && ok; ++dz)
      for (int dy = -1; dy <= 1 && ok; ++dy)
        for (int dx = -1; dx <= 1 && ok; ++dx) {
          if (!dx && !dy && !dz) continue;
          int64_t q[3] = {p[0] + dx, p[1] + dy, p[2] + dz};
          if (!t.inside(L - 1, q[0], q[1], q[2])) continue;  // beyond a wall
          int lc;
          if (t.at(L - 1, q[0], q[1], q[2]) >= 0 || t.coarser(L - 1, q[0], q[1], q[2], &lc) >= 0) continue;
          const int del[3] = {dx, dy, dz};
          for (int c = 0; c < 8 && ok; ++c) {
            const int o[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
            bool touch = true;
            for (int e = 0; e < 3; ++e)
              if ((del[e] < 0 && o[e] == 0) || (del[e] > 0 && o[e] == 1)) touch = false;
            if (!touch) continue;
            const int32_t cid = t.at(L, 2 * q[0] + o[0], 2 * q[1] + o[1], 2 * q[2] + o[2]);
            if (cid < 0 || ref[cid]) ok = false;
          }
        }
    if (ok)
      for (int c = 0; c < 8; ++c) der[sib[c]] = c == 0 ? 2 : 1;
  }
  bool any = false;
  for (int64_t b = 0; b < nl; ++b) any |= ref[b] || der[b];
  std::fill(m->flags.begin(), m->flags.end(), 0);
  if (!any) return PKH_OK;
  // new leaves with their source: kind 0 copy, 1 child, 2 merged parent
  struct NewLeaf {
    pkh_loc loc;
    int32_t kind, src;
  };
  std::vector<NewLeaf> nv;
  for (int64_t b = 0; b < nl; ++b) {
    const pkh_loc& l = t.leaves[b];
    if (ref[b]) {
      for (int c = 0; c < 8; ++c)
        nv.push_back({{l.level + 1, 2 * l.lx1 + (c & 1), 2 * l.lx2 + ((c >> 1) & 1), 2 * l.lx3 + ((c >> 2) & 1)},
                      1, (int32_t)b});
    } else if (der[b] == 2) {
      nv.push_back({{l.level - 1, l.lx1 >> 1, l.lx2 >> 1, l.lx3 >> 1}, 2, (int32_t)b});
    } else if (der[b] == 0) {
      nv.push_back({l, 0, (int32_t)b});
    }
  }
  Tree nt;
  std::copy(t.nrb, t.nrb + 3, nt.nrb);
  std::copy(t.periodic, t.periodic + 3, nt.periodic);
  nt.maxl = t.maxl;
  std::stable_sort(nv.begin(), nv.end(), [&](const NewLeaf& a, const NewLeaf& b) {
    uint64_t ka = t.key(a.loc), kb = t.key(b.loc);
    return ka != kb ? ka < kb : a.loc.level < b.loc.level;
  });
  for (auto& x : nv) nt.leaves.push_back(x.loc);
  int rc = nt.build();
  if (rc) return rc;
  // device: new state from the old one
  std::vector<int32_t> kind(nv.size()), src(nv.size());
  for (size_t r = 0; r < nv.size(); ++r) {
    kind[r] = nv[r].kind;
    src[r] = nv[r].src;
  }
  drop_graph(m);
  double* oldA = m->A;
  double* oldB = m->B;
  BlockInfo* old_blocks = m->d_blocks;
  int32_t* old_map = m->d_map;
  LevelMaps old_maps = m->maps;
  m->d_blocks = nullptr;
  m->d_map = nullptr;
  free_cycle_tables(m);
  m->tree = std::move(nt);
  int32_t *d_kind = nullptr, *d_src = nullptr;
  if ((rc = build_tables(m, m->h_blocks, &m->d_map, m->maps)) || (rc = alloc_state(m, false)) ||
      (rc = upload_vec(m, &d_kind, kind)) || (rc = upload_vec(m, &d_src, src)))
    return rc;
  HIPCHK(launch_regrid_data(m->A, m->d_blocks, d_kind, d_src, (int32_t)m->nb(), oldA, old_blocks,
                            old_maps, m->g, m->d_time, m->stream));
  // frees are ordered after the regrid kernel on the stream (or, with
  // hipFree, synchronise by themselves)
  m->dfree(d_kind);
  m->dfree(d_src);
  m->state_free(oldA);
  m->state_free(oldB);
  m->dfree(old_blocks);
  m->dfree(old_map);
  m->flags.assign(m->nb(), 0);
  if ((rc = ensure_partials(m))) return rc;
  // the ghost faces the cycle and the indicators read (level jumps, walls,
  // remote faces; same-level halos are read from the neighbours), then the
  // new state's CFL timestep
  if (m->njf) HIPCHK(launch_fill_faces(m->A, m->g, m->d_time, m->d_jf, m->d_plan, m->njf, m->stream));
  if ((rc = exchange_remote(m, m->A, false))) return rc;
  if ((rc = refresh_dt(m))) return rc;
  m->ghosts_valid = true;
  return check_err(m);
}

int pkh_conserved_totals(pkh_mesh* m, double out[5]) {
  if (!m || !out) return fail(PKH_EINVAL, "null argument");
  if (m->fp32)
    HIPCHK(launch_totals(m->d_partial, m->d_tot, m->Af(), m->d_blocks, (int32_t)m->nb(), m->g, m->stream));
  else
    HIPCHK(launch_totals(m->d_partial, m->d_tot, m->A, m->d_blocks, (int32_t)m->nb(), m->g, m->stream));
  HIPCHK(hipMemcpyAsync(out, m->d_tot, NV * sizeof(double), hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return check_err(m);
}

int pkh_conserved_totals_noalloc(pkh_mesh* m, double out[5]) {
  if (!m || !out) return fail(PKH_EINVAL, "null argument");
  if (m->nb() > TOTALS_SCRATCH_LEAVES)
    return fail(PKH_EINVAL, "%lld leaves exceed the %d the static totals scratch holds; use pkh_conserved_totals",
                (long long)m->nb(), TOTALS_SCRATCH_LEAVES);
  double* scr = nullptr;
  HIPCHK(totals_scratch(m->device, &scr));
  if (m->fp32)
    HIPCHK(launch_totals_scratch(m->Af(), m->d_blocks, (int32_t)m->nb(), m->g, scr, m->stream));
  else
    HIPCHK(launch_totals_scratch(m->A, m->d_blocks, (int32_t)m->nb(), m->g, scr, m->stream));
  HIPCHK(hipMemcpyAsync(out, scr + (int64_t)TOTALS_SCRATCH_LEAVES * NV, NV * sizeof(double),
                        hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return check_err(m);
}

int pkh_set_tuning(pkh_mesh* m, const pkh_tuning* t) {
  if (!m || !t) return fail(PKH_EINVAL, "null argument");
  if (m->fp32 && t->tile_rows != 0 && t->tile_rows != 8 && t->tile_rows != 16)
    return fail(PKH_EINVAL, "FP32 state storage takes tile_rows 0, 8 or 16");
  if (stage_tile_rows(m->g.n1, m->g.n2, t->tile_rows) < 0)
    return fail(PKH_EINVAL, "tile_rows %d not available for blocks of %d x %d", t->tile_rows, m->g.n1,
                m->g.n2);
  if (t->packs < 0) return fail(PKH_EINVAL, "packs must be >= 0");
  const int32_t packs = std::max<int32_t>(1, t->packs);
  if (t->tile_rows != m->tj || packs != m->packs) drop_graph(m);
  m->tj = t->tile_rows;
  m->packs = packs;
  return PKH_OK;
}

int pkh_set_partition(pkh_mesh* m, int32_t nparts) {
  if (!m) return fail(PKH_EINVAL, "null mesh");
  if (nparts < 1 || nparts > m->nb()) return fail(PKH_EINVAL, "nparts must be in [1, %lld]", (long long)m->nb());
  if (m->fp32 && nparts > 1) return fail(PKH_EINVAL, "partitions need an FP64-stored state");
  if (nparts == m->nparts) return PKH_OK;
  if (m->attached)
    return fail(PKH_ESTATE, "%d tape(s) or batch(es) hold this mesh's layout; destroy them before repartitioning",
                m->attached);
  HIPCHK(hipStreamSynchronize(m->stream));  // queued work may use the tables
  drop_graph(m);
  m->nparts = nparts;
  free_tables(m);
  int rc;
  if ((rc = build_tables(m, m->h_blocks, &m->d_map, m->maps))) return rc;
  // ghost layers of faces that just became remote were never written by the
  // direct-read path: fill them from the current state
  if ((rc = exchange_remote(m, m->A, false))) return rc;
  HIPCHK(hipStreamSynchronize(m->stream));
  return PKH_OK;
}

int pkh_get_partition(const pkh_mesh* m, int32_t* nparts, int32_t* nremote, int32_t* nmessages) {
  if (!m) return fail(PKH_EINVAL, "null mesh");
  if (nparts) *nparts = m->nparts;
  if (nremote) *nremote = m->nrf;
  if (nmessages) *nmessages = (int32_t)m->msgs.size();
  return PKH_OK;
}

int pkh_get_tuning(const pkh_mesh* m, pkh_tuning* t) {
  if (!m || !t) return fail(PKH_EINVAL, "null argument");
  *t = pkh_tuning{};
  t->tile_rows = stage_tile_rows(m->g.n1, m->g.n2, m->tj, m->nb());
  t->packs = m->packs;
  return PKH_OK;
}

int pkh_kernel_timing(pkh_mesh* m, uint32_t kinds) {
  if (!m) return fail(PKH_EINVAL, "null mesh");
  HIPCHK(hipStreamSynchronize(m->stream));
  m->kt_mask = kinds & 63u;
  m->kt_rec.clear();
  m->ev_used = 0;
  return PKH_OK;
}

int pkh_kernel_times(pkh_mesh* m, double* ms, int64_t* count) {
  if (!m || !ms || !count) return fail(PKH_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(m->stream));
  for (int k = 0; k < PKH_KT_KINDS; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
  }
  for (const auto& r : m->kt_rec) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, m->ev_pool[r[1]], m->ev_pool[r[2]]));
    ms[r[0]] += t;
    count[r[0]] += 1;
  }
  return PKH_OK;
}

// ---------------------------------------------------------------------------
// Reverse mode
// ---------------------------------------------------------------------------
}  // extern "C"

struct pkh_tape {
  pkh_mesh* m = nullptr;
  int32_t K = 1;                 // checkpoint interval
  int32_t ncycles = 0;           // recorded cycles
  std::vector<double*> ckpt;     // active-layout states at cycles 0, K, 2K, ...
  double* d_dts = nullptr;       // dt of every recorded cycle
  int32_t dts_cap = 0;
  std::vector<double*> S;        // recomputed ghost-filled U^n, K + 1 of them
  std::vector<double*> Us;       // recomputed ghost-filled U*, K of them
  double* wbar = nullptr;        // padded primitive-adjoint scratch for y and z
  double* xlast = nullptr;       // parts across x faces, 20 doubles per row
  double* lam[3] = {nullptr, nullptr, nullptr};  // active-layout adjoints
  DevTime* d_time = nullptr;     // clock for recomputation (dt from the record)
  // face-wise reverse (meshes with level jumps or walls; optional otherwise):
  // one padded adjoint scratch instead of the pencil and row buffers
  bool facewise = false;
  double* gw = nullptr;
};

namespace {
size_t active_bytes(const pkh_mesh* m) {
  return (size_t)m->nb() * NV * m->g.n1 * m->g.n2 * m->g.n3 * sizeof(double);
}

void tape_free(pkh_tape* t) {
  pkh_mesh* m = t->m;
  for (double* p : t->ckpt) m->dfree(p);
  for (double* p : t->S) m->padded_free(p);
  for (double* p : t->Us) m->padded_free(p);
  t->ckpt.clear();
  t->S.clear();
  t->Us.clear();
  m->dfree(t->d_dts);
  m->padded_free(t->wbar);
  m->dfree(t->xlast);
  m->padded_free(t->gw);
  t->gw = nullptr;
  for (auto& l : t->lam) m->dfree(l);
  m->dfree(t->d_time);
  t->d_dts = nullptr;
  t->wbar = nullptr;
  t->xlast = nullptr;
  t->d_time = nullptr;
  for (auto& l : t->lam) l = nullptr;
}

// Ghost-filled recomputation of cycle inputs S[0..len] and U*[0..len-1]
// from the checkpoint of a segment starting at cycle c0.
int tape_recompute(pkh_tape* t, int c0, int len) {
  pkh_mesh* m = t->m;
  const int32_t nb = (int32_t)m->nb();
  HIPCHK(launch_scatter(t->S[0], t->ckpt[c0 / t->K], nb, m->g, m->stream));
  HIPCHK(launch_fill(t->S[0], m->d_blocks, nb, m->g, m->maps, t->d_time, 0, m->stream));
  StageLaunch s{};
  s.blocks = m->d_blocks;
  s.nblocks = nb;
  s.g = m->g;
  s.tm = t->d_time;
  s.fbuf = m->d_fbuf;
  s.nbr = m->d_nbr;
  s.tj = m->tj;
  s.do_dt = 0;
  // the level-jump and wall work of a stage on its output, as in the cycle
  auto level_jumps = [&](double* u, double beta) -> hipError_t {
    if (m->ncblocks) {
      const hipError_t e = launch_flux_correct(u, m->d_blocks, m->d_ff, m->d_ff_first, m->d_cblocks, m->ncblocks,
                                               m->g, t->d_time, beta, 0, m->d_fbuf, m->d_nbr, m->stream);
      if (e != hipSuccess) return e;
    }
    if (m->njf) return launch_fill_faces(u, m->g, t->d_time, m->d_jf, m->d_plan, m->njf, m->stream);
    return hipSuccess;
  };
  for (int q = 0; q < len; ++q) {
    HIPCHK(launch_tape_dt(t->d_time, t->d_dts, c0 + q, 0, m->stream));
    s.uin = t->S[q];
    s.ubase = t->S[q];
    s.uout = t->Us[q];
    s.beta = 0.5;
    s.recon = m->cfg.stage1_recon;
    HIPCHK(launch_stage(s, m->stream));
    HIPCHK(level_jumps(t->Us[q], 0.5));
    s.uin = t->Us[q];
    s.ubase = t->S[q];
    s.uout = t->S[q + 1];
    s.beta = 1.0;
    s.recon = PKH_RECON_PLM;
    HIPCHK(launch_stage(s, m->stream));
    HIPCHK(level_jumps(t->S[q + 1], 1.0));
  }
  return PKH_OK;
}
}  // namespace

extern "C" {

int pkh_tape_create(pkh_mesh* m, int32_t ckpt_every, pkh_tape** out) {
  if (!m || !out || ckpt_every < 1) return fail(PKH_EINVAL, "bad argument");
  *out = nullptr;
  if (m->fp32 || m->nparts > 1)
    return fail(PKH_EINVAL, "the reverse mode needs an FP64-stored mesh without a partition");
  pkh_tape* t = new pkh_tape();
  t->m = m;
  t->K = ckpt_every;
  // level jumps or walls: the face-wise reverse; blocks the row kernels do
  // not cover: the same
  t->facewise = m->need_fill || m->ncblocks || !adj_xrow_supported(m->g.n1);
  const size_t pb = m->state_bytes();
  bool ok = true;
  for (int q = 0; q <= ckpt_every && ok; ++q) {
    t->S.push_back(m->padded_alloc(pb));
    ok = t->S.back() != nullptr;
  }
  for (int q = 0; q < ckpt_every && ok; ++q) {
    t->Us.push_back(m->padded_alloc(pb));
    ok = t->Us.back() != nullptr;
  }
  if (ok) {
    if (t->facewise) {
      t->gw = m->padded_alloc(pb);
    } else {
      t->wbar = m->padded_alloc(2 * pb);
      t->xlast = (double*)m->dalloc((size_t)m->nb() * m->g.n2 * m->g.n3 * 20 * sizeof(double));
    }
    for (auto& l : t->lam) l = (double*)m->dalloc(active_bytes(m));
    t->d_time = (DevTime*)m->dalloc(sizeof(DevTime));
    ok = (t->facewise ? t->gw != nullptr : (t->wbar && t->xlast)) && t->lam[0] && t->lam[1] && t->lam[2] &&
         t->d_time;
  }
  if (!ok) {
    tape_free(t);
    delete t;
    return fail(PKH_ENOMEM, "tape allocation failed");
  }
  // ghost zones of the recomputation buffers start defined
  for (double* p : t->S) HIPCHK(hipMemsetAsync(p, 0, pb, m->stream));
  for (double* p : t->Us) HIPCHK(hipMemsetAsync(p, 0, pb, m->stream));
  HIPCHK(hipMemcpyAsync(t->d_time, m->d_time, sizeof(DevTime), hipMemcpyDeviceToDevice, m->stream));
  m->attached++;
  *out = t;
  return PKH_OK;
}

int pkh_tape_destroy(pkh_tape* t) {
  if (!t) return PKH_OK;
  (void)hipStreamSynchronize(t->m->stream);
  tape_free(t);
  t->m->attached--;
  delete t;
  return PKH_OK;
}

int pkh_tape_set_facewise(pkh_tape* t, int32_t on) {
  if (!t) return fail(PKH_EINVAL, "null tape");
  pkh_mesh* m = t->m;
  const bool need = m->need_fill || m->ncblocks || !adj_xrow_supported(m->g.n1);
  if (!on && need) return fail(PKH_EINVAL, "this mesh needs the face-wise reverse");
  if ((on != 0) == t->facewise) return PKH_OK;
  HIPCHK(hipStreamSynchronize(m->stream));
  const size_t pb = m->state_bytes();
  m->padded_free(t->gw);
  m->padded_free(t->wbar);
  m->dfree(t->xlast);
  t->gw = t->wbar = t->xlast = nullptr;
  t->facewise = on != 0;
  if (t->facewise) {
    t->gw = m->padded_alloc(pb);
    if (!t->gw) return fail(PKH_ENOMEM, "tape allocation failed");
  } else {
    t->wbar = m->padded_alloc(2 * pb);
    t->xlast = (double*)m->dalloc((size_t)m->nb() * m->g.n2 * m->g.n3 * 20 * sizeof(double));
    if (!t->wbar || !t->xlast) return fail(PKH_ENOMEM, "tape allocation failed");
  }
  return PKH_OK;
}

int pkh_forward_taped(pkh_mesh* m, pkh_tape* t, int32_t n) {
  if (!m || !t || t->m != m || n < 1) return fail(PKH_EINVAL, "bad argument");
  int rc;
  if (!m->ghosts_valid && (rc = do_exchange(m))) return rc;
  const int nck = (n + t->K - 1) / t->K;
  HIPCHK(hipStreamSynchronize(m->stream));
  for (double* p : t->ckpt) m->dfree(p);
  t->ckpt.clear();
  for (int q = 0; q < nck; ++q) {
    t->ckpt.push_back((double*)m->dalloc(active_bytes(m)));
    if (!t->ckpt.back()) return fail(PKH_ENOMEM, "checkpoint allocation failed");
  }
  if (t->dts_cap < n) {
    m->dfree(t->d_dts);
    t->d_dts = (double*)m->dalloc((size_t)n * sizeof(double));
    if (!t->d_dts) return fail(PKH_ENOMEM, "allocation failed");
    t->dts_cap = n;
  }
  t->ncycles = n;
  HIPCHK(launch_clock(m->d_time, CLOCK_BEGIN, INFINITY, m->stream));
  for (int c = 0; c < n; ++c) {
    if (c % t->K == 0) HIPCHK(launch_gather(t->ckpt[c / t->K], m->A, (int32_t)m->nb(), m->g, m->stream));
    HIPCHK(launch_tape_dt(m->d_time, t->d_dts, c, 1, m->stream));
    if ((rc = enqueue_cycle(m, c + 1 < n ? (CLOCK_END | CLOCK_BEGIN) : CLOCK_END, INFINITY))) return rc;
  }
  return PKH_OK;
}

int pkh_tape_replay(pkh_mesh* m, pkh_tape* t) {
  if (!m || !t || t->m != m) return fail(PKH_EINVAL, "bad argument");
  if (t->ncycles < 1) return fail(PKH_ESTATE, "nothing recorded on the tape");
  int rc;
  if (!m->ghosts_valid && (rc = do_exchange(m))) return rc;
  for (int c = 0; c < t->ncycles; ++c) {
    HIPCHK(launch_tape_dt(m->d_time, t->d_dts, c, 0, m->stream));
    if ((rc = enqueue_cycle(m, CLOCK_END, INFINITY))) return rc;
  }
  return PKH_OK;
}

int pkh_adjoint(pkh_mesh* m, pkh_tape* t, const double* lam_final, double* grad_init) {
  if (!m || !t || t->m != m || !lam_final || !grad_init) return fail(PKH_EINVAL, "bad argument");
  if (t->ncycles < 1) return fail(PKH_ESTATE, "nothing recorded on the tape");
  const int32_t nb = (int32_t)m->nb();
  int rc;
  double* lam = t->lam[0];
  double* lam_star = t->lam[1];
  double* lam_new = t->lam[2];
  HIPCHK(hipMemcpyAsync(lam, lam_final, active_bytes(m), hipMemcpyDeviceToDevice, m->stream));
  const int nseg = (t->ncycles + t->K - 1) / t->K;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int c0 = seg * t->K;
    const int len = std::min(t->K, t->ncycles - c0);
    if ((rc = tape_recompute(t, c0, len))) return rc;
    for (int q = len - 1; q >= 0; --q) {
      const double* dtp = t->d_dts + c0 + q;
      if (t->facewise) {
        {
          KTimer kt(m, 4, false);
          HIPCHK(launch_adj_stage_facewise(PKH_RECON_PLM, t->Us[q], lam, t->gw, m->d_blocks, nb, m->g, m->d_nbr,
                                           m->maps, m->d_jf, m->njf, dtp, 1.0, lam_star, nullptr, nullptr,
                                           m->d_time, m->stream));
        }
        {
          KTimer kt(m, 4, false);
          HIPCHK(launch_adj_stage_facewise(m->cfg.stage1_recon, t->S[q], lam_star, t->gw, m->d_blocks, nb, m->g,
                                           m->d_nbr, m->maps, m->d_jf, m->njf, dtp, 0.5, lam_new, lam, lam_star,
                                           m->d_time, m->stream));
        }
        std::swap(lam, lam_new);
        continue;
      }
      {  // corrector: lam* = (dU^{n+1}/dU*)^T lam
        KTimer kt(m, 4, false);
        HIPCHK(launch_adj_stage(PKH_RECON_PLM, t->Us[q], lam, t->wbar, t->xlast, m->d_blocks, nb, m->g, m->d_nbr,
                                dtp, 1.0, lam_star, nullptr, nullptr, m->stream));
      }
      {  // predictor and the identities: lam^n = lam + lam* + (dU*/dU^n)^T-term of lam*
        KTimer kt(m, 4, false);
        HIPCHK(launch_adj_stage(m->cfg.stage1_recon, t->S[q], lam_star, t->wbar, t->xlast, m->d_blocks, nb, m->g,
                                m->d_nbr, dtp, 0.5, lam_new, lam, lam_star, m->stream));
      }
      std::swap(lam, lam_new);
    }
  }
  HIPCHK(hipMemcpyAsync(grad_init, lam, active_bytes(m), hipMemcpyDeviceToDevice, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  t->lam[0] = lam;
  t->lam[2] = lam_new;
  return check_err(m);
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
}  // extern "C"

struct pkh_batch {
  std::vector<pkh_mesh*> meshes;
  hipStream_t stream = nullptr;
  struct Group {
    int n1 = 0, tj = 0;
    std::vector<int32_t> members;   // mesh indices
    std::vector<GroupItem> items;
    GroupItem* d_items = nullptr;
  };
  std::vector<Group> groups;
  StageLaunch* d_pred = nullptr;    // per mesh: predictor launch parameters
  StageLaunch* d_corr = nullptr;    // per mesh: corrector launch parameters
  DevTime** d_tms = nullptr;        // per mesh clock
  hipGraphExec_t gexec = nullptr;
  int32_t g_cycles = 0;
  // persistent launch: instance descriptors, progress counters, the items
  // of one cycle, ticket counter and error word
  bool p_ok = false;                // every mesh has blocks of 16 or 32 cells per row
  PInst* d_pinst = nullptr;
  PSync* d_psync = nullptr;
  PItem* d_pitems = nullptr;
  PCtl* d_pctl = nullptr;           // per XCD slot
  int32_t* d_slot_of = nullptr;     // XCD id -> slot
  int32_t nslots = 0;
  int32_t npitems = 0;              // items of one cycle over all slots
  int32_t pwaves = 2;               // waves per SIMD of the persistent kernel (2 or 3)
  double wait_limit_s = 2.0;        // bound of every wait inside the persistent kernel
  int32_t wall_khz = 0;             // device wall-clock rate
  bool attached = false;            // counted in every member's attached count
};

namespace {
void batch_drop_graph(pkh_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
  b->g_cycles = 0;
}

void batch_free_items(pkh_batch* b) {
  pkh_mesh* m0 = b->meshes[0];
  for (auto& gr : b->groups) {
    m0->dfree(gr.d_items);
    gr.d_items = nullptr;
  }
}

// Work items of each group for its current tile rows (block-major, tiles of
// a block consecutive).
int batch_build_items(pkh_batch* b) {
  pkh_mesh* m0 = b->meshes[0];
  batch_free_items(b);
  batch_drop_graph(b);
  for (auto& gr : b->groups) {
    gr.items.clear();
    for (int32_t mi : gr.members) {
      pkh_mesh* m = b->meshes[mi];
      m->tj = gr.tj;
      for (int32_t blk = 0; blk < (int32_t)m->nb(); ++blk)
        for (int32_t j0 = 0; j0 < m->g.n2; j0 += gr.tj) gr.items.push_back(GroupItem{mi, blk, j0, 0});
    }
    int rc = upload_vec(m0, &gr.d_items, gr.items);
    if (rc) return rc;
  }
  HIPCHK(hipStreamSynchronize(b->stream));
  return PKH_OK;
}

// The level-jump work of one stage of every multilevel mesh: flux
// correction, then the ghost faces across level jumps and walls.
int batch_level_jumps(pkh_batch* b, bool corrector) {
  for (pkh_mesh* m : b->meshes) {
    double* u = corrector ? m->A : m->B;
    if (m->ncblocks)
      HIPCHK(launch_flux_correct(u, m->d_blocks, m->d_ff, m->d_ff_first, m->d_cblocks, m->ncblocks, m->g,
                                 m->d_time, corrector ? 1.0 : 0.5, corrector ? 1 : 0, m->d_fbuf, m->d_nbr,
                                 b->stream));
    if (m->njf) HIPCHK(launch_fill_faces(u, m->g, m->d_time, m->d_jf, m->d_plan, m->njf, b->stream));
  }
  return PKH_OK;
}

int batch_enqueue_cycle(pkh_batch* b, int mode_after) {
  int rc;
  for (const auto& gr : b->groups)
    HIPCHK(launch_stage_group(b->meshes[gr.members[0]]->cfg.stage1_recon, gr.n1, gr.tj, b->d_pred, gr.d_items,
                              (int)gr.items.size(), b->stream));
  if ((rc = batch_level_jumps(b, false))) return rc;
  for (const auto& gr : b->groups)
    HIPCHK(launch_stage_group(PKH_RECON_PLM, gr.n1, gr.tj, b->d_corr, gr.d_items, (int)gr.items.size(),
                              b->stream));
  if ((rc = batch_level_jumps(b, true))) return rc;
  HIPCHK(launch_clock_group(b->d_tms, (int32_t)b->meshes.size(), mode_after, INFINITY, b->stream));
  return PKH_OK;
}

int batch_prepare(pkh_batch* b) {
  int rc;
  for (pkh_mesh* m : b->meshes)
    if (!m->ghosts_valid && (rc = do_exchange(m))) return rc;
  return PKH_OK;
}

int batch_fused(pkh_batch* b, int32_t n, bool graph) {
  int rc;
  if ((rc = batch_prepare(b))) return rc;
  HIPCHK(launch_clock_group(b->d_tms, (int32_t)b->meshes.size(), CLOCK_BEGIN, INFINITY, b->stream));
  int c = 0;
  if (graph) {
    const int K = std::min(n, 50);
    if (!b->gexec || b->g_cycles != K) {
      batch_drop_graph(b);
      hipGraph_t gh = nullptr;
      HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      for (int q = 0; q < K && !rc; ++q) rc = batch_enqueue_cycle(b, CLOCK_END | CLOCK_BEGIN);
      hipError_t e = hipStreamEndCapture(b->stream, &gh);
      if (rc) return rc;
      if (e != hipSuccess) return fail(PKH_EHIP, "graph capture failed: %s", hipGetErrorString(e));
      e = hipGraphInstantiate(&b->gexec, gh, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gh);
      if (e != hipSuccess) return fail(PKH_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
      b->g_cycles = K;
    }
    for (; c + K <= n; c += K) HIPCHK(hipGraphLaunch(b->gexec, b->stream));
  }
  for (; c < n; ++c)
    if ((rc = batch_enqueue_cycle(b, CLOCK_END | CLOCK_BEGIN))) return rc;
  return PKH_OK;
}

// Descriptors and items of the persistent launch. The XCDs the device runs
// workgroups on are found by a probe launch; each instance is pinned to one
// of them (largest instances first, each to the least loaded XCD by cells),
// and each XCD's items are ordered by phase, then instance (largest first).
int batch_build_persistent(pkh_batch* b, const std::vector<StageLaunch>& pred,
                           const std::vector<StageLaunch>& corr) {
  pkh_mesh* m0 = b->meshes[0];
  const int32_t n = (int32_t)b->meshes.size();
  int32_t seen[PMAX_XCC] = {};
  int32_t* d_probe = (int32_t*)m0->dalloc(PMAX_XCC * sizeof(int32_t));
  if (!d_probe) return fail(PKH_ENOMEM, "persistent batch allocation failed");
  const hipError_t pe = probe_xcc(d_probe, seen, b->stream);
  m0->dfree(d_probe);
  if (pe != hipSuccess) return fail(PKH_EHIP, "XCD probe failed: %s", hipGetErrorString(pe));
  std::vector<int32_t> slot_of(PMAX_XCC, -1);
  int32_t nslots = 0;
  for (int x = 0; x < PMAX_XCC; ++x)
    if (seen[x]) slot_of[x] = nslots++;
  if (nslots < 1) return fail(PKH_EHIP, "XCD probe saw no workgroup");
  auto cells = [&](int32_t q) {
    const pkh_mesh* m = b->meshes[q];
    return m->nb() * m->g.n1 * m->g.n2 * m->g.n3;
  };
  std::vector<int32_t> order(n);
  for (int32_t q = 0; q < n; ++q) order[q] = q;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cells(x) > cells(y); });
  std::vector<int64_t> load(nslots, 0);
  std::vector<std::vector<int32_t>> members(nslots);
  for (int32_t q : order) {
    int best = 0;
    for (int k = 1; k < nslots; ++k)
      if (load[k] < load[best]) best = k;
    load[best] += cells(q);
    members[best].push_back(q);
  }
  std::vector<PInst> pin(n);
  std::vector<PItem> items;
  std::vector<PCtl> ctl(nslots);
  for (int k = 0; k < nslots; ++k) {
    std::vector<PItem> per[PPHASES];
    for (int32_t q : members[k]) {
      pkh_mesh* m = b->meshes[q];
      PInst& pi = pin[q];
      pi = PInst{};
      pi.st[0] = pred[q];
      pi.st[1] = corr[q];
      pi.ff = m->d_ff;
      pi.ff_first = m->d_ff_first;
      pi.cblocks = m->d_cblocks;
      pi.jf = m->d_jf;
      pi.plan = m->d_plan;
      pi.n1 = m->g.n1;
      const int tj = persistent_tile_rows(m->g.n1);
      for (int32_t blk = 0; blk < (int32_t)m->nb(); ++blk)
        for (int32_t j0 = 0; j0 < m->g.n2; j0 += tj) {
          per[0].push_back(PItem{q, 0, blk, j0});
          per[3].push_back(PItem{q, 3, blk, j0});
        }
      pi.cnt[0] = pi.cnt[3] = (int32_t)(m->nb() * (m->g.n2 / tj));
      const int nshell = 2 * m->g.n1 * m->g.n2 + (m->g.n3 - 2) * (2 * m->g.n1 + 2 * (m->g.n2 - 2));
      const int nfc = (nshell + 255) / 256;
      for (int32_t c = 0; c < m->ncblocks; ++c)
        for (int32_t x = 0; x < nfc; ++x) {
          per[1].push_back(PItem{q, 1, x, c});
          per[4].push_back(PItem{q, 4, x, c});
        }
      pi.cnt[1] = pi.cnt[4] = m->ncblocks * nfc;
      const int nff = fill_faces_stride(m->g) / 256;
      for (int32_t f = 0; f < m->njf; ++f)
        for (int32_t x = 0; x < nff; ++x) {
          per[2].push_back(PItem{q, 2, x, f});
          per[5].push_back(PItem{q, 5, x, f});
        }
      pi.cnt[2] = pi.cnt[5] = m->njf * nff;
      pi.last = pi.cnt[5] ? 5 : (pi.cnt[4] ? 4 : 3);
    }
    ctl[k] = PCtl{};
    ctl[k].off = (int32_t)items.size();
    for (auto& v : per) items.insert(items.end(), v.begin(), v.end());
    ctl[k].nper = (int32_t)items.size() - ctl[k].off;
  }
  b->npitems = (int32_t)items.size();
  b->nslots = nslots;
  int rc;
  if ((rc = upload_vec(m0, &b->d_pinst, pin)) || (rc = upload_vec(m0, &b->d_pitems, items)) ||
      (rc = upload_vec(m0, &b->d_pctl, ctl)) || (rc = upload_vec(m0, &b->d_slot_of, slot_of)))
    return rc;
  b->d_psync = (PSync*)m0->dalloc(n * sizeof(PSync));
  if (!b->d_psync) return fail(PKH_ENOMEM, "persistent batch allocation failed");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&b->wall_khz, hipDeviceAttributeWallClockRate, dev));
  return PKH_OK;
}

// n cycles of every instance by persistent launches of up to 50 cycles each.
int batch_persistent(pkh_batch* b, int32_t n) {
  if (!b->p_ok) return fail(PKH_EINVAL, "the persistent launch takes blocks of 16 or 32 cells per row only");
  int rc;
  if ((rc = batch_prepare(b))) return rc;
  const int grid = (int)std::min<int64_t>(persistent_grid(b->pwaves), (int64_t)b->npitems * std::min(n, 50));
  if (grid < 1) return fail(PKH_EHIP, "persistent kernel occupancy query failed");
  const long long ticks = (long long)(b->wait_limit_s * 1e3 * (double)b->wall_khz);
  HIPCHK(launch_clock_group(b->d_tms, (int32_t)b->meshes.size(), CLOCK_BEGIN, INFINITY, b->stream));
  for (int c = 0; c < n; c += 50) {
    const int K = std::min(50, n - c);
    HIPCHK(launch_persistent(b->d_pinst, (int32_t)b->meshes.size(), b->d_psync, b->d_pitems, b->d_slot_of,
                             b->d_pctl, b->nslots, K, b->pwaves, grid, ticks, b->stream));
  }
  return PKH_OK;
}

// Save / restore of the active state and clock of every mesh (autotuning).
struct Saved {
  std::vector<double*> A;
  std::vector<DevTime*> tm;
};

int save_states(const std::vector<pkh_mesh*>& ms, Saved& sv) {
  for (pkh_mesh* m : ms) {
    double* a = (double*)m->dalloc(m->state_bytes());
    DevTime* t = (DevTime*)m->dalloc(sizeof(DevTime));
    if (!a || !t) return fail(PKH_ENOMEM, "autotune scratch allocation failed");
    HIPCHK(hipMemcpyAsync(a, m->A, m->state_bytes(), hipMemcpyDeviceToDevice, m->stream));
    HIPCHK(hipMemcpyAsync(t, m->d_time, sizeof(DevTime), hipMemcpyDeviceToDevice, m->stream));
    sv.A.push_back(a);
    sv.tm.push_back(t);
  }
  return PKH_OK;
}

int restore_states(const std::vector<pkh_mesh*>& ms, Saved& sv) {
  for (size_t q = 0; q < ms.size(); ++q) {
    pkh_mesh* m = ms[q];
    HIPCHK(hipMemcpyAsync(m->A, sv.A[q], m->state_bytes(), hipMemcpyDeviceToDevice, m->stream));
    HIPCHK(hipMemcpyAsync(m->d_time, sv.tm[q], sizeof(DevTime), hipMemcpyDeviceToDevice, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    m->dfree(sv.A[q]);
    m->dfree(sv.tm[q]);
  }
  return PKH_OK;
}

const int kTileChoices[] = {4, 8, 16, 2};
}  // namespace

extern "C" {

int pkh_batch_create(pkh_mesh* const* meshes, int32_t n, const pkh_tuning* tuning, pkh_batch** out) {
  if (!meshes || n < 1 || !out) return fail(PKH_EINVAL, "bad argument");
  *out = nullptr;
  for (int32_t q = 0; q < n; ++q)
    for (int32_t r = 0; r < q; ++r)
      if (meshes[q] == meshes[r]) return fail(PKH_EINVAL, "a mesh appears twice in the batch");
  pkh_batch* b = new pkh_batch();
  b->meshes.assign(meshes, meshes + n);
  b->stream = meshes[0] ? meshes[0]->stream : nullptr;
  b->p_ok = true;
  for (pkh_mesh* m : b->meshes) {
    if (!m || m->stream != b->stream) {
      delete b;
      return fail(PKH_EINVAL, "batched meshes must share one stream");
    }
    if (m->fp32 || m->nparts > 1) {
      delete b;
      return fail(PKH_EINVAL, "batches hold FP64-stored meshes without a partition");
    }
    if (tuning && tuning->tile_rows) {
      if (stage_tile_rows(m->g.n1, m->g.n2, tuning->tile_rows) != tuning->tile_rows) {
        delete b;
        return fail(PKH_EINVAL, "tile_rows %d not available for blocks of %d x %d", tuning->tile_rows, m->g.n1,
                    m->g.n2);
      }
      m->tj = tuning->tile_rows;
    }
    b->p_ok &= persistent_tile_rows(m->g.n1) > 0 && m->g.n2 % persistent_tile_rows(m->g.n1) == 0;
  }
  std::vector<StageLaunch> pred(n), corr(n);
  std::vector<DevTime*> tms(n);
  for (int32_t q = 0; q < n; ++q) {
    pkh_mesh* m = b->meshes[q];
    StageLaunch s{};
    s.blocks = m->d_blocks;
    s.nblocks = (int32_t)m->nb();
    s.g = m->g;
    s.tm = m->d_time;
    s.fbuf = m->d_fbuf;
    s.nbr = m->d_nbr;
    s.uin = m->A;
    s.ubase = m->A;
    s.uout = m->B;
    s.beta = 0.5;
    s.recon = m->cfg.stage1_recon;
    s.do_dt = 0;
    pred[q] = s;
    s.uin = m->B;
    s.uout = m->A;
    s.beta = 1.0;
    s.recon = PKH_RECON_PLM;
    s.do_dt = 1;
    corr[q] = s;
    tms[q] = m->d_time;
    // group by block width and stage-1 reconstruction
    const int tj = stage_tile_rows(m->g.n1, m->g.n2, m->tj, m->nb());
    bool placed = false;
    for (auto& gr : b->groups) {
      pkh_mesh* r = b->meshes[gr.members[0]];
      if (gr.n1 == m->g.n1 && r->cfg.stage1_recon == m->cfg.stage1_recon &&
          stage_tile_rows(m->g.n1, m->g.n2, gr.tj) == gr.tj) {
        gr.members.push_back(q);
        placed = true;
        break;
      }
    }
    if (!placed) {
      pkh_batch::Group gr;
      gr.n1 = m->g.n1;
      gr.tj = tj;
      gr.members.push_back(q);
      b->groups.push_back(gr);
    }
  }
  pkh_mesh* m0 = b->meshes[0];
  int rc;
  if ((rc = upload_vec(m0, &b->d_pred, pred)) || (rc = upload_vec(m0, &b->d_corr, corr)) ||
      (rc = upload_vec(m0, &b->d_tms, tms)) || (rc = batch_build_items(b)) ||
      (b->p_ok && (rc = batch_build_persistent(b, pred, corr)))) {
    pkh_batch_destroy(b);
    return rc;
  }
  for (pkh_mesh* m : b->meshes) m->attached++;
  b->attached = true;
  *out = b;
  return PKH_OK;
}

int pkh_batch_destroy(pkh_batch* b) {
  if (!b) return PKH_OK;
  (void)hipStreamSynchronize(b->stream);
  batch_drop_graph(b);
  batch_free_items(b);
  pkh_mesh* m0 = b->meshes[0];
  m0->dfree(b->d_pred);
  m0->dfree(b->d_corr);
  m0->dfree(b->d_tms);
  m0->dfree(b->d_pinst);
  m0->dfree(b->d_psync);
  m0->dfree(b->d_pitems);
  m0->dfree(b->d_pctl);
  m0->dfree(b->d_slot_of);
  if (b->attached)
    for (pkh_mesh* m : b->meshes) m->attached--;
  delete b;
  return PKH_OK;
}

int pkh_batch_step(pkh_batch* b, int32_t n, uint32_t mode) {
  if (!b || n < 0 || mode > PKH_PERSISTENT) return fail(PKH_EINVAL, "bad argument");
  if (n == 0) return PKH_OK;
  if (mode == PKH_PLAIN) {
    int rc;
    for (int c = 0; c < n; ++c)
      for (pkh_mesh* m : b->meshes)
        if ((rc = pkh_step(m, 1, INFINITY))) return rc;
    return PKH_OK;
  }
  if (mode == PKH_PERSISTENT) return batch_persistent(b, n);
  return batch_fused(b, n, mode == PKH_GRAPH);
}

int pkh_batch_set_tuning(pkh_batch* b, const pkh_batch_tuning* t) {
  if (!b || !t) return fail(PKH_EINVAL, "null argument");
  if (t->waves_per_simd != 0 && t->waves_per_simd != 2 && t->waves_per_simd != 3)
    return fail(PKH_EINVAL, "waves_per_simd must be 0, 2 or 3");
  if (!(t->wait_limit_s >= 0.0) || t->wait_limit_s > 3600.0)
    return fail(PKH_EINVAL, "wait_limit_s must be in [0, 3600]");
  b->pwaves = t->waves_per_simd ? t->waves_per_simd : 2;
  b->wait_limit_s = t->wait_limit_s > 0.0 ? t->wait_limit_s : 0.0;
  return PKH_OK;
}

int pkh_batch_get_tuning(const pkh_batch* b, pkh_batch_tuning* t) {
  if (!b || !t) return fail(PKH_EINVAL, "null argument");
  *t = pkh_batch_tuning{};
  t->waves_per_simd = b->pwaves;
  t->wait_limit_s = b->wait_limit_s;
  return PKH_OK;
}

int pkh_batch_autotune(pkh_batch* b, int32_t trial_cycles, int32_t* tile_rows) {
  if (!b || trial_cycles < 1) return fail(PKH_EINVAL, "bad argument");
  int rc;
  if ((rc = batch_prepare(b))) return rc;
  Saved sv;
  if ((rc = save_states(b->meshes, sv))) return rc;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (auto& gr : b->groups) {
    int best = gr.tj;
    float best_ms = 1e30f;
    for (int tj : kTileChoices) {
      if (stage_tile_rows(gr.n1, b->meshes[gr.members[0]]->g.n2, tj) != tj) continue;
      bool all = true;
      for (int32_t mi : gr.members) all &= stage_tile_rows(gr.n1, b->meshes[mi]->g.n2, tj) == tj;
      if (!all) continue;
      gr.tj = tj;
      if ((rc = batch_build_items(b))) return rc;
      if ((rc = batch_fused(b, 1, false))) return rc;  // warm-up
      HIPCHK(hipEventRecord(e0, b->stream));
      if ((rc = batch_fused(b, trial_cycles, false))) return rc;
      HIPCHK(hipEventRecord(e1, b->stream));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) {
        best_ms = ms;
        best = tj;
      }
    }
    gr.tj = best;
  }
  if (b->p_ok) {  // waves per SIMD of the persistent kernel
    int best = b->pwaves;
    float best_ms = 1e30f;
    for (int w : {2, 3}) {
      b->pwaves = w;
      if ((rc = batch_persistent(b, 1))) return rc;  // warm-up
      HIPCHK(hipEventRecord(e0, b->stream));
      if ((rc = batch_persistent(b, trial_cycles))) return rc;
      HIPCHK(hipEventRecord(e1, b->stream));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) {
        best_ms = ms;
        best = w;
      }
    }
    b->pwaves = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if ((rc = batch_build_items(b)) || (rc = restore_states(b->meshes, sv))) return rc;
  if (tile_rows)
    for (size_t q = 0; q < b->meshes.size(); ++q) tile_rows[q] = stage_tile_rows(b->meshes[q]->g.n1, b->meshes[q]->g.n2, b->meshes[q]->tj);
  return PKH_OK;
}

int pkh_autotune(pkh_mesh* m, int32_t trial_cycles, pkh_tuning* out) {
  if (!m || trial_cycles < 1) return fail(PKH_EINVAL, "bad argument");
  int rc;
  if (!m->ghosts_valid && (rc = do_exchange(m))) return rc;
  std::vector<pkh_mesh*> ms{m};
  Saved sv;
  if ((rc = save_states(ms, sv))) return rc;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const uint32_t flags = m->cfg.flags;
  m->cfg.flags &= ~PKH_FLAG_GRAPH;
  int best = stage_tile_rows(m->g.n1, m->g.n2, m->tj, m->nb());
  float best_ms = 1e30f;
  for (int tj : kTileChoices) {
    if (stage_tile_rows(m->g.n1, m->g.n2, tj) != tj) continue;
    if (m->fp32 && tj != 8 && !(m->g.n1 == 32 && tj == 16)) continue;
    m->tj = tj;
    if ((rc = pkh_step(m, 1, INFINITY))) break;
    HIPCHK(hipEventRecord(e0, m->stream));
    if ((rc = pkh_step(m, trial_cycles, INFINITY))) break;
    HIPCHK(hipEventRecord(e1, m->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = tj;
    }
  }
  m->cfg.flags = flags;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  m->tj = best;
  drop_graph(m);
  int rc2 = restore_states(ms, sv);
  if (rc) return rc;
  if (rc2) return rc2;
  if (out) {
    *out = pkh_tuning{};
    out->tile_rows = best;
    out->packs = m->packs;
  }
  return PKH_OK;
}

int pkh_sync(pkh_mesh* m) {
  if (!m) return fail(PKH_EINVAL, "null mesh");
  return check_err(m);
}

}  // extern "C"
