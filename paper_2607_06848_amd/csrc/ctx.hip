// Context creation, integer tables and small host-side API of the EFE library.
//
// Integer tables (node, cell and local numbering, colours, boundary, support
// lists of the enrichment and projector functions, their node-major
// transposes) are built here on the host; every floating-point quantity of
// the method is computed by the kernels in setup.hip and the other sources.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "efe_internal.h"

efe_status efe_alloc(efe_ctx *ctx, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
    return EFE_ENOMEM;
  }
  return EFE_OK;
}

efe_status efe_ws(efe_ctx *ctx, int slot, size_t bytes, void **p) {
  if (ctx->arena) {
    // no allocation: the slot gets (or has) a fixed place in the arena
    if (slot < 0 || slot >= efe_ctx::kArenaSlots) EFE_FAIL(ctx, EFE_EINVAL, "bad scratch slot");
    if (ctx->arena_len[slot] == 0) {
      const size_t off = (ctx->arena_used + 255) & ~(size_t)255;
      if (off + bytes > ctx->arena_cap)
        EFE_FAIL(ctx, EFE_EINVAL, "the scratch region is too small for this call");
      ctx->arena_off[slot] = off;
      ctx->arena_len[slot] = std::max<size_t>(bytes, 1);
      ctx->arena_used = off + ctx->arena_len[slot];
    } else if (ctx->arena_len[slot] < bytes) {
      EFE_FAIL(ctx, EFE_EINVAL, "a scratch slot grew within one call");
    }
    *p = ctx->arena + ctx->arena_off[slot];
    return EFE_OK;
  }
  if ((int)ctx->ws.size() <= slot) ctx->ws.resize(slot + 1);
  DevBuf &b = ctx->ws[slot];
  if (b.bytes < bytes) {
    if (b.p) {
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      HIPCHK(ctx, hipFree(b.p));
    }
    b.p = nullptr;
    b.bytes = 0;
    efe_status s = efe_alloc(ctx, &b.p, bytes);
    if (s) return s;
    b.bytes = bytes;
  }
  *p = b.p;
  return EFE_OK;
}

template <class T>
static efe_status upload(efe_ctx *ctx, T **dst, const std::vector<T> &src) {
  efe_status s = efe_alloc(ctx, (void **)dst, src.size() * sizeof(T));
  if (s) return s;
  if (!src.empty())
    HIPCHK(ctx, hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice,
                               ctx->stream));
  return EFE_OK;
}

// message of the last failed efe_setup_mesh on this thread
static thread_local std::string g_setup_error;

void efe_set_global_error(const std::string &msg) { g_setup_error = msg; }

// --------------------------------------------------------------- mesh tables
static void build_mesh_tables(efe_ctx *c) {
  const int P = c->P, p = c->p;
  const int64_t n1x = c->n1[0], n1y = c->n1[1];
  c->c2g.resize((size_t)c->n_cells * c->nloc);
  for (int64_t cid = 0; cid < c->n_cells; ++cid) {
    int64_t cx = cid % c->ncell[0], cy = (cid / c->ncell[0]) % c->ncell[1],
            cz = cid / ((int64_t)c->ncell[0] * c->ncell[1]);
    for (int l = 0; l < c->nloc; ++l) {
      int a = l % P, b = (l / P) % P, cc = l / (P * P);
      int64_t gi = cx * p + a, gj = cy * p + b, gk = cz * p + cc;
      c->c2g[cid * c->nloc + l] = (int32_t)(gi + n1x * (gj + n1y * gk));
    }
  }
  std::vector<int> colour(c->n_cells);
  for (int64_t cid = 0; cid < c->n_cells; ++cid) {
    int64_t cx = cid % c->ncell[0], cy = (cid / c->ncell[0]) % c->ncell[1],
            cz = cid / ((int64_t)c->ncell[0] * c->ncell[1]);
    colour[cid] = (int)((cx & 1) + 2 * (cy & 1) + 4 * (cz & 1));
  }
  c->colour_order.clear();
  for (int col = 0; col < 8; ++col) {
    c->colour_offsets[col] = (int32_t)c->colour_order.size();
    for (int64_t cid = 0; cid < c->n_cells; ++cid)
      if (colour[cid] == col) c->colour_order.push_back((int32_t)cid);
  }
  c->colour_offsets[8] = (int32_t)c->colour_order.size();
  c->boundary.assign(c->n_nodes, 0);
  for (int64_t n = 0; n < c->n_nodes; ++n) {
    int64_t i = n % n1x, j = (n / n1x) % n1y, k = n / (n1x * n1y);
    if (i == 0 || i == c->n1[0] - 1 || j == 0 || j == c->n1[1] - 1 || k == 0 ||
        k == c->n1[2] - 1)
      c->boundary[n] = 1;
  }
}

// Cells whose box distance to `x` is below rc: sum over axes of
// max(0, lo - x, x - hi)^2, lo = box_lo + c h, hi = box_lo + (c+1) h, summed
// x, then y, then z, without contraction, so the table is reproducible.
static void support_cells(const efe_ctx *c, const double *x, double rc,
                          std::vector<int32_t> &out) {
#pragma clang fp contract(off)
  std::vector<double> t2[3];
  for (int d = 0; d < 3; ++d) {
    t2[d].resize(c->ncell[d]);
    for (int i = 0; i < c->ncell[d]; ++i) {
      double lo = c->lo[d] + (double)i * c->h[d];
      double hi = c->lo[d] + ((double)i + 1.0) * c->h[d];
      double t = std::max(std::max(lo - x[d], x[d] - hi), 0.0);
      t2[d][i] = t * t;
    }
  }
  const double r2 = rc * rc;
  for (int64_t cid = 0; cid < c->n_cells; ++cid) {
    int64_t cx = cid % c->ncell[0], cy = (cid / c->ncell[0]) % c->ncell[1],
            cz = cid / ((int64_t)c->ncell[0] * c->ncell[1]);
    double s = t2[0][cx] + t2[1][cy];
    s = s + t2[2][cz];
    if (s < r2) out.push_back((int32_t)cid);
  }
}

// Support nodes (interior nodes of the support cells, ascending) of every
// atom, the per-pair local-to-support map and the node-major transpose.
struct SupportTables {
  std::vector<int32_t> ptr, cells, pair_atom, pair_cell, lmap, snode_ptr, snode, nm_ptr, nm_atom,
      nm_src;
};

static void build_support(const efe_ctx *c, double rc, SupportTables &T) {
  T.ptr.assign(c->natoms + 1, 0);
  for (int I = 0; I < c->natoms; ++I) {
    support_cells(c, &c->xyz[3 * I], rc, T.cells);
    T.ptr[I + 1] = (int32_t)T.cells.size();
  }
  const int64_t np = (int64_t)T.cells.size();
  T.pair_atom.resize(np);
  T.pair_cell = T.cells;
  for (int I = 0; I < c->natoms; ++I)
    for (int32_t q = T.ptr[I]; q < T.ptr[I + 1]; ++q) T.pair_atom[q] = I;
  // support nodes per atom
  T.snode_ptr.assign(c->natoms + 1, 0);
  std::vector<int32_t> mark(c->n_nodes, -1);
  T.lmap.assign((size_t)np * c->nloc, -1);
  for (int I = 0; I < c->natoms; ++I) {
    std::vector<int32_t> nodes;
    for (int32_t q = T.ptr[I]; q < T.ptr[I + 1]; ++q) {
      const int32_t *g = &c->c2g[(size_t)T.cells[q] * c->nloc];
      for (int l = 0; l < c->nloc; ++l)
        if (!c->boundary[g[l]] && mark[g[l]] != I) {
          mark[g[l]] = I;
          nodes.push_back(g[l]);
        }
    }
    std::sort(nodes.begin(), nodes.end());
    const int32_t base = (int32_t)T.snode.size();
    T.snode.insert(T.snode.end(), nodes.begin(), nodes.end());
    T.snode_ptr[I + 1] = (int32_t)T.snode.size();
    for (int32_t q = T.ptr[I]; q < T.ptr[I + 1]; ++q) {
      const int32_t *g = &c->c2g[(size_t)T.cells[q] * c->nloc];
      for (int l = 0; l < c->nloc; ++l) {
        if (c->boundary[g[l]]) continue;
        auto it = std::lower_bound(nodes.begin(), nodes.end(), g[l]);
        T.lmap[(size_t)q * c->nloc + l] = base + (int32_t)(it - nodes.begin());
      }
    }
  }
  // node-major: per node the atoms (ascending) whose support holds it
  T.nm_ptr.assign(c->n_nodes + 1, 0);
  for (int I = 0; I < c->natoms; ++I)
    for (int32_t s = T.snode_ptr[I]; s < T.snode_ptr[I + 1]; ++s) T.nm_ptr[T.snode[s] + 1]++;
  for (int64_t n = 0; n < c->n_nodes; ++n) T.nm_ptr[n + 1] += T.nm_ptr[n];
  T.nm_atom.resize(T.nm_ptr[c->n_nodes]);
  T.nm_src.resize(T.nm_ptr[c->n_nodes]);
  std::vector<int32_t> fill(T.nm_ptr.begin(), T.nm_ptr.end() - 1);
  for (int I = 0; I < c->natoms; ++I)
    for (int32_t s = T.snode_ptr[I]; s < T.snode_ptr[I + 1]; ++s) {
      int32_t e = fill[T.snode[s]]++;
      T.nm_atom[e] = I;
      T.nm_src[e] = s;
    }
}

// Work items of the atom-major reductions over support nodes: every atom's
// (node-sorted) support list cut at multiples of `region` node indices and
// at `maxlen` entries, as (atom, first, end) triples.  Region r goes to XCD
// r % 8 (round robin keeps the dense middle of a cluster spread over all
// XCDs) and each XCD's items are stored together, region by region, so that
// the items of a region run on one XCD and re-read its rows from that XCD's
// L2.  items_off[x] .. items_off[x+1] are XCD x's items.
static void build_items(int natoms, int64_t n_nodes, const std::vector<int32_t> &ptr,
                        const std::vector<int32_t> &snode, int32_t region, int32_t maxlen,
                        std::vector<int32_t> &items, int64_t items_off[9]) {
  struct It { int32_t reg, atom, s0, s1; };
  std::vector<It> v;
  for (int I = 0; I < natoms; ++I) {
    int32_t s = ptr[I];
    while (s < ptr[I + 1]) {
      const int32_t reg = snode[s] / region;
      int32_t e = s + 1;
      while (e < ptr[I + 1] && e - s < maxlen && snode[e] / region == reg) ++e;
      v.push_back({reg, I, s, e});
      s = e;
    }
  }
  (void)n_nodes;
  std::stable_sort(v.begin(), v.end(), [](const It &a, const It &b) {
    return a.reg % 8 != b.reg % 8 ? a.reg % 8 < b.reg % 8 : a.reg < b.reg;
  });
  items.clear();
  size_t k = 0;
  for (int x = 0; x < 8; ++x) {
    items_off[x] = (int64_t)items.size() / 3;
    for (; k < v.size() && v[k].reg % 8 == x; ++k) {
      items.push_back(v[k].atom);
      items.push_back(v[k].s0);
      items.push_back(v[k].s1);
    }
  }
  items_off[8] = (int64_t)items.size() / 3;
}

// (cell, I, J) for every cell and every pair of atoms from lists A and B whose
// supports contain the cell.
static void build_triples(const efe_ctx *c, const SupportTables &A, const SupportTables &B,
                          std::vector<int32_t> &trip) {
  std::vector<std::vector<int32_t>> ca(c->n_cells), cb(c->n_cells);
  for (size_t q = 0; q < A.pair_cell.size(); ++q) ca[A.pair_cell[q]].push_back(A.pair_atom[q]);
  for (size_t q = 0; q < B.pair_cell.size(); ++q) cb[B.pair_cell[q]].push_back(B.pair_atom[q]);
  for (int64_t cid = 0; cid < c->n_cells; ++cid)
    for (int32_t I : ca[cid])
      for (int32_t J : cb[cid]) {
        trip.push_back((int32_t)cid);
        trip.push_back(I);
        trip.push_back(J);
      }
}

// ------------------------------------------------------------------- API
extern "C" efe_status efe_setup_mesh(const efe_mesh_desc *mesh, const efe_system_desc *sys,
                                     void *stream, efe_ctx **out) {
  if (!out) return EFE_EINVAL;
  *out = nullptr;
  if (!mesh || !sys) return EFE_EINVAL;
  if (mesh->p < 1 || mesh->p > EFE_MAXP || mesh->nq < 1 || mesh->nq > EFE_MAXQ) return EFE_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (mesh->ncell[d] < 1 || !(mesh->hi[d] > mesh->lo[d])) return EFE_EINVAL;
  if (sys->natoms < 0 || (sys->natoms > 0 && (!sys->xyz || !sys->Z))) return EFE_EINVAL;
  if (sys->enr_lmax > 2) return EFE_EINVAL;
  const bool tab = sys->enr_lmax >= 0 && sys->enr_tab_n > 0;
  if (sys->enr_lmax >= 0 && !(sys->enr_rcut > 0 && sys->enr_t > 0 && (tab || sys->enr_alpha > 0)))
    return EFE_EINVAL;
  if (sys->atom_tab_n > 0) {
    if (!sys->atom_tab || sys->atom_tab_n < 2 || !(sys->atom_tab_dr > 0)) return EFE_EINVAL;
    for (int I = 1; I < sys->natoms; ++I)
      if (sys->Z[I] != sys->Z[0]) return EFE_EINVAL;   // one species
  }
  if (tab) {
    if (!sys->enr_tab || sys->enr_tab_n < 2 || !(sys->enr_tab_dr > 0)) return EFE_EINVAL;
    for (int l = 0; l <= sys->enr_lmax; ++l)
      if (!(sys->enr_tab_rc[l] > 0) || sys->enr_tab_rc[l] > sys->enr_rcut) return EFE_EINVAL;
  }
  if (sys->kb_width > 0 && !(sys->kb_rcut > 0)) return EFE_EINVAL;
  if (!(sys->loc_rc > 0) || !(sys->loc_rg > 0)) return EFE_EINVAL;

  efe_ctx *c = new efe_ctx();
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return EFE_EHIP;
  }
  for (int d = 0; d < 3; ++d) {
    c->lo[d] = mesh->lo[d];
    c->hi[d] = mesh->hi[d];
    c->ncell[d] = mesh->ncell[d];
    c->h[d] = (c->hi[d] - c->lo[d]) / (double)c->ncell[d];
    c->n1[d] = (int64_t)c->ncell[d] * mesh->p + 1;
  }
  c->p = mesh->p;
  c->P = mesh->p + 1;
  c->nloc = c->P * c->P * c->P;
  c->nq = mesh->nq;
  c->nqp = c->nq * c->nq * c->nq;
  c->n_nodes = c->n1[0] * c->n1[1] * c->n1[2];
  c->n_cells = (int64_t)c->ncell[0] * c->ncell[1] * c->ncell[2];
  c->n_qpts = c->n_cells * c->nqp;
  if (c->n_nodes > INT32_MAX / 2 || c->n_cells * c->nloc > INT32_MAX) {
    delete c;
    return EFE_EINVAL;
  }
  c->natoms = sys->natoms;
  c->xyz.assign(sys->xyz, sys->xyz + 3 * (size_t)sys->natoms);
  c->Z.assign(sys->Z, sys->Z + (size_t)sys->natoms);
  c->loc_rc = sys->loc_rc;
  c->loc_amp = sys->loc_amp;
  c->loc_rg = sys->loc_rg;
  c->kb_width = sys->kb_width;
  c->kb_D = sys->kb_D;
  c->kb_rcut = sys->kb_rcut;
  c->lmax = sys->enr_lmax;
  c->enr_alpha = sys->enr_alpha;
  c->enr_rcut = sys->enr_rcut;
  c->enr_t = sys->enr_t;
  c->rho_alpha = sys->rho_alpha;
  if (tab) {
    c->ntab = sys->enr_tab_n;
    c->tab_dr = sys->enr_tab_dr;
    for (int l = 0; l <= sys->enr_lmax; ++l) c->tab_rc[l] = sys->enr_tab_rc[l];
    c->tab_host.assign(sys->enr_tab, sys->enr_tab + (size_t)2 * (sys->enr_lmax + 1) * c->ntab);
  }
  if (sys->atom_tab_n > 0) {
    c->natab = sys->atom_tab_n;
    c->atab_dr = sys->atom_tab_dr;
    c->atab_host.assign(sys->atom_tab, sys->atom_tab + (size_t)4 * c->natab);
  }
  c->nf = c->lmax < 0 ? 0 : (c->lmax + 1) * (c->lmax + 1);
  if (c->natoms == 0) c->nf = 0;
  c->n_enr = (int64_t)c->natoms * c->nf;
  c->nproj = (c->kb_width > 0 && c->kb_D != 0 && c->natoms > 0) ? c->natoms : 0;
  c->rows = c->n_nodes + c->n_enr;

  build_mesh_tables(c);
  int64_t nb = 0;
  for (auto b : c->boundary) nb += b;
  c->n_dof = c->n_nodes - nb + c->n_enr;

  efe_status s = EFE_OK;
#define TRY(x)            \
  do {                    \
    s = (x);              \
    if (s) goto fail;     \
  } while (0)
  {
    TRY(upload(c, &c->d_c2g, c->c2g));
    TRY(upload(c, &c->d_colour_order, c->colour_order));
    std::vector<double> xyz = c->xyz, Zs = c->Z;
    TRY(upload(c, &c->d_xyz, xyz));
    TRY(upload(c, &c->d_Zs, Zs));
    if (c->ntab > 0) TRY(upload(c, &c->d_enr_tab, c->tab_host));
    if (c->natab > 0) TRY(upload(c, &c->d_atom_tab, c->atab_host));
    TRY(efe_build_reference(c));

    SupportTables E, K;
    if (c->nf > 0) build_support(c, c->enr_rcut, E);
    else E.ptr.assign(c->natoms + 1, 0), E.snode_ptr.assign(c->natoms + 1, 0),
         E.nm_ptr.assign(c->n_nodes + 1, 0);
    if (c->nproj > 0) build_support(c, c->kb_rcut, K);
    else K.ptr.assign(c->natoms + 1, 0), K.snode_ptr.assign(c->natoms + 1, 0),
         K.nm_ptr.assign(c->n_nodes + 1, 0);
    c->enr_ptr = E.ptr;
    c->enr_cells = E.cells;
    c->kb_ptr = K.ptr;
    c->kb_cells = K.cells;
    c->npairs = (int64_t)E.cells.size();
    c->n_snodes = (int64_t)E.snode.size();
    c->snode_ptr_h = E.snode_ptr;
    c->nnz_nm = (int64_t)E.nm_atom.size();
    TRY(upload(c, &c->d_pair_atom, E.pair_atom));
    TRY(upload(c, &c->d_pair_cell, E.pair_cell));
    TRY(upload(c, &c->d_pair_lmap, E.lmap));
    TRY(upload(c, &c->d_snode_ptr, E.snode_ptr));
    TRY(upload(c, &c->d_snode, E.snode));
    TRY(upload(c, &c->d_nm_ptr, E.nm_ptr));
    TRY(upload(c, &c->d_nm_atom, E.nm_atom));
    TRY(upload(c, &c->d_nm_src, E.nm_src));
    // groups of 8 consecutive nodes: union of their atoms, and per node-major
    // entry the slot of its atom in its group's union
    {
      const int64_t G = cdiv(c->n_nodes, 8);
      std::vector<int32_t> gptr(G + 1, 0), gatom, gslot(E.nm_atom.size());
      std::vector<int32_t> u;
      for (int64_t gi = 0; gi < G; ++gi) {
        const int64_t n0 = gi * 8, n1 = std::min<int64_t>(n0 + 8, c->n_nodes);
        u.assign(E.nm_atom.begin() + E.nm_ptr[n0], E.nm_atom.begin() + E.nm_ptr[n1]);
        std::sort(u.begin(), u.end());
        u.erase(std::unique(u.begin(), u.end()), u.end());
        for (int64_t n = n0; n < n1; ++n)
          for (int32_t e = E.nm_ptr[n]; e < E.nm_ptr[n + 1]; ++e)
            gslot[e] = (int32_t)gatom.size() +
                       (int32_t)(std::lower_bound(u.begin(), u.end(), E.nm_atom[e]) - u.begin());
        gatom.insert(gatom.end(), u.begin(), u.end());
        gptr[gi + 1] = (int32_t)gatom.size();
      }
      c->n_gslots = (int64_t)gatom.size();
      TRY(upload(c, &c->d_g_ptr, gptr));
      TRY(upload(c, &c->d_g_atom, gatom));
      TRY(upload(c, &c->d_nm_gslot, gslot));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    // coupling pairs: per atom every cell that holds one of its support nodes
    // (its support cells and the layer of cells around them, where C is
    // non-zero on shared nodes although phi vanishes), with the local-to-
    // support map and the support pair of the cell (-1 for the outer layer);
    // then their cell-major view (atom-major pairs are sorted by atom, so a
    // cell's pairs come out in ascending atom order)
    {
      std::vector<int32_t> cptr(c->natoms + 1, 0), catom, ccell, cspair, clmap;
      std::vector<int32_t> pos(c->n_nodes, -1), cmark(c->n_cells, -1);
      const int64_t n1x = c->n1[0], n1y = c->n1[1];
      for (int I = 0; I < c->natoms && c->nf > 0; ++I) {
        std::vector<int32_t> cl;
        for (int32_t sI = E.snode_ptr[I]; sI < E.snode_ptr[I + 1]; ++sI) {
          const int64_t nd = E.snode[sI];
          pos[nd] = sI;
          const int64_t ijk[3] = {nd % n1x, (nd / n1x) % n1y, nd / (n1x * n1y)};
          int cs[3][2], nc[3];
          for (int d = 0; d < 3; ++d) {
            const int cc = (int)(ijk[d] / c->p), aa = (int)(ijk[d] % c->p);
            nc[d] = 0;
            if (aa == 0 && cc > 0) cs[d][nc[d]++] = cc - 1;
            if (cc < c->ncell[d]) cs[d][nc[d]++] = cc;
          }
          for (int z = 0; z < nc[2]; ++z)
            for (int y = 0; y < nc[1]; ++y)
              for (int x = 0; x < nc[0]; ++x) {
                const int32_t cell =
                    cs[0][x] + c->ncell[0] * (cs[1][y] + c->ncell[1] * cs[2][z]);
                if (cmark[cell] != I) {
                  cmark[cell] = I;
                  cl.push_back(cell);
                }
              }
        }
        std::sort(cl.begin(), cl.end());
        for (int32_t cell : cl) {
          catom.push_back(I);
          ccell.push_back(cell);
          auto it = std::lower_bound(E.cells.begin() + E.ptr[I], E.cells.begin() + E.ptr[I + 1],
                                     cell);
          cspair.push_back(it != E.cells.begin() + E.ptr[I + 1] && *it == cell
                               ? (int32_t)(it - E.cells.begin())
                               : -1);
          const int32_t *gl = &c->c2g[(size_t)cell * c->nloc];
          for (int l = 0; l < c->nloc; ++l) clmap.push_back(c->boundary[gl[l]] ? -1 : pos[gl[l]]);
        }
        cptr[I + 1] = (int32_t)catom.size();
        for (int32_t sI = E.snode_ptr[I]; sI < E.snode_ptr[I + 1]; ++sI) pos[E.snode[sI]] = -1;
      }
      c->ncpairs = (int64_t)catom.size();
      std::vector<int32_t> eptr(c->n_cells + 1, 0), epair(ccell.size()), cpos(ccell.size());
      for (int32_t cc : ccell) eptr[cc + 1]++;
      for (int64_t cc = 0; cc < c->n_cells; ++cc) eptr[cc + 1] += eptr[cc];
      std::vector<int32_t> fill(eptr.begin(), eptr.end() - 1);
      for (size_t q = 0; q < ccell.size(); ++q) {
        const int32_t at = fill[ccell[q]]++;
        epair[at] = (int32_t)q;
        cpos[q] = at;
      }
      std::vector<int64_t> noff(c->n_cells + 1, 0);
      int maxr = 0;
      for (int64_t cc = 0; cc < c->n_cells; ++cc) {
        const int64_t ne = (int64_t)(eptr[cc + 1] - eptr[cc]) * c->nf;
        const int64_t nep = (ne + 15) / 16 * 16;
        noff[cc + 1] = noff[cc] + nep;
        maxr = std::max<int>(maxr, (int)(nep / 16));
      }
      c->max_rbe = maxr;
      c->n_epad = noff[c->n_cells];
      if ((int64_t)maxr * 16 > EFE_MAX_CELL_ENR) {
        c->err = "more than " + std::to_string(EFE_MAX_CELL_ENR) +
                 " enrichment functions couple to one cell";
        s = EFE_EINVAL;
        goto fail;
      }
      TRY(upload(c, &c->d_cpair_atom, catom));
      TRY(upload(c, &c->d_cpair_spair, cspair));
      TRY(upload(c, &c->d_cpair_lmap, clmap));
      TRY(upload(c, &c->d_cpair_ptr, cptr));
      TRY(upload(c, &c->d_cell_eptr, eptr));
      TRY(upload(c, &c->d_cell_epair, epair));
      TRY(upload(c, &c->d_cpair_cpos, cpos));
      TRY(upload(c, &c->d_cell_noff, noff));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    std::vector<int32_t> items;
    build_items(c->natoms, c->n_nodes, E.snode_ptr, E.snode, 512, 1024, items, c->enr_items_off);
    c->n_enr_items = (int64_t)items.size() / 3;
    TRY(upload(c, &c->d_enr_items, items));
    std::vector<int32_t> trip;
    if (c->nf > 0) build_triples(c, E, E, trip);
    c->ntrip = (int64_t)trip.size() / 3;
    TRY(upload(c, &c->d_trip, trip));

    c->nkbpairs = (int64_t)K.cells.size();
    c->n_kbnodes = (int64_t)K.snode.size();
    c->nnz_kbnm = (int64_t)K.nm_atom.size();
    TRY(upload(c, &c->d_kbpair_atom, K.pair_atom));
    TRY(upload(c, &c->d_kbpair_cell, K.pair_cell));
    TRY(upload(c, &c->d_kbpair_lmap, K.lmap));
    TRY(upload(c, &c->d_kbnode_ptr, K.snode_ptr));
    TRY(upload(c, &c->d_kbnode, K.snode));
    TRY(upload(c, &c->d_kbnm_ptr, K.nm_ptr));
    TRY(upload(c, &c->d_kbnm_atom, K.nm_atom));
    TRY(upload(c, &c->d_kbnm_src, K.nm_src));
    std::vector<int32_t> kbitems;
    build_items(c->natoms, c->n_nodes, K.snode_ptr, K.snode, 512, 1024, kbitems, c->kb_items_off);
    c->n_kb_items = (int64_t)kbitems.size() / 3;
    TRY(upload(c, &c->d_kb_items, kbitems));
    std::vector<int32_t> kbtrip;
    if (c->nproj > 0 && c->nf > 0) build_triples(c, K, E, kbtrip);
    c->nkbtrip = (int64_t)kbtrip.size() / 3;
    TRY(upload(c, &c->d_kbtrip, kbtrip));
    HIPCHK(c, hipStreamSynchronize(c->stream));   // host vectors go out of scope
    TRY(efe_build_enrichment(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    TRY(efe_scratch_attach(c));
  }
#undef TRY
  *out = c;
  return EFE_OK;
fail:
  g_setup_error = c->err;
  efe_destroy(c);
  return s;
}

extern "C" efe_status efe_enrichment_amplification(const efe_ctx *c, double *amp) {
  if (!c || !amp) return EFE_EINVAL;
  *amp = c->amplification;
  return EFE_OK;
}

extern "C" efe_status efe_get_coupling(const efe_ctx *c, int64_t *ncpairs, int64_t *max_cell) {
  if (!c) return EFE_EINVAL;
  if (ncpairs) *ncpairs = c->ncpairs;
  if (max_cell) *max_cell = (int64_t)c->max_rbe * 16;
  return EFE_OK;
}

extern "C" efe_status efe_get_sizes(const efe_ctx *c, int64_t *s) {
  if (!c || !s) return EFE_EINVAL;
  s[0] = c->rows;
  s[1] = c->n_nodes;
  s[2] = c->n_dof;
  s[3] = c->n_enr;
  s[4] = c->n_cells;
  s[5] = c->n_qpts;
  s[6] = c->natoms;
  s[7] = c->nloc;
  return EFE_OK;
}

extern "C" efe_status efe_get_tables(const efe_ctx *c, int32_t *c2g, int32_t *order,
                                     int32_t *offsets, uint8_t *boundary) {
  if (!c) return EFE_EINVAL;
  if (c2g) memcpy(c2g, c->c2g.data(), c->c2g.size() * sizeof(int32_t));
  if (order) memcpy(order, c->colour_order.data(), c->colour_order.size() * sizeof(int32_t));
  if (offsets) memcpy(offsets, c->colour_offsets, 9 * sizeof(int32_t));
  if (boundary) memcpy(boundary, c->boundary.data(), c->boundary.size());
  return EFE_OK;
}

extern "C" efe_status efe_get_support(const efe_ctx *c, int32_t which, int64_t *npairs,
                                      int32_t *ptr, int32_t *cells) {
  if (!c || !npairs || (which != 0 && which != 1)) return EFE_EINVAL;
  const std::vector<int32_t> &P = which == 0 ? c->enr_ptr : c->kb_ptr;
  const std::vector<int32_t> &C = which == 0 ? c->enr_cells : c->kb_cells;
  *npairs = (int64_t)C.size();
  if (ptr) memcpy(ptr, P.data(), P.size() * sizeof(int32_t));
  if (cells && !C.empty()) memcpy(cells, C.data(), C.size() * sizeof(int32_t));
  return EFE_OK;
}

extern "C" const char *efe_last_error(const efe_ctx *c) {
  return c ? c->err.c_str() : g_setup_error.c_str();
}

extern "C" void efe_destroy(efe_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  efe_scf_free(c);
  void *ptrs[] = {c->d_c2g,       c->d_colour_order, c->d_m,          c->d_minv, c->d_m_int,
                  c->d_N3,        c->d_G3,           c->d_W3,         c->d_K,
                  c->d_xq1,       c->d_xyz,          c->d_Zs,         c->d_pair_atom,
                  c->d_pair_cell, c->d_pair_lmap,    c->d_snode_ptr,  c->d_snode,
                  c->d_nu,        c->d_b_am,         c->d_C_am,       c->d_Bkin_am,
                  c->d_B_am,      c->d_nm_ptr,       c->d_nm_atom,    c->d_nm_src,
                  c->d_trip,      c->d_Mpp,
                  c->d_Mee,       c->d_Hpp_kin,      c->d_Hpp,        c->d_Mee_inv,
                  c->d_kbpair_atom, c->d_kbpair_cell, c->d_kbpair_lmap, c->d_kbnode_ptr,
                  c->d_kbnode,    c->d_Pc_am,        c->d_kbnm_ptr,   c->d_kbnm_atom,
                  c->d_kbnm_src,  c->d_Pc_nm,        c->d_kbtrip,     c->d_Pphi,
                  c->d_D,         c->d_vq,           c->d_Htile64,    c->d_Htile32,
                  c->d_Htile16,   c->d_enr_items,    c->d_kb_items,   c->d_g_ptr,
                  c->d_g_atom,    c->d_nm_gslot,     c->d_Cg,         c->d_Bg,
                  c->d_cell_eptr, c->d_cell_epair,   c->d_cpair_cpos, c->d_cell_noff,
                  c->d_Bkin_pair, c->d_B_pair,       c->d_Et64,       c->d_Ee64,
                  c->d_Et32,      c->d_Ee32,         c->d_Hee,
                  c->d_Ptil,      c->d_cpair_ptr,    c->d_cpair_atom, c->d_cpair_spair,
                  c->d_cpair_lmap};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (auto &b : c->ws)
    if (b.p) (void)hipFree(b.p);
  for (auto &v : c->tev)
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
  delete c;
}
