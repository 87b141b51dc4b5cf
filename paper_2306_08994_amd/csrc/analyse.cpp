// analyse.cpp -- host analysis: nested-dissection elimination tree, Foata classes, pivot and
// contribution-block sets, front index lists, extend-add maps and the launch schedule.
//
// Tree (Sec. 2.4, Table 3): the leaves are the element matrices and fronts are joined pairwise
// into a binary tree that follows the mesh.  With element coordinates the pairing is recursive
// coordinate bisection of the element index box: split the axis holding the most elements
// (ties: the lowest axis) at lo + floor(len/2), lower half first, down to single elements.
// Without them (connectivity only) it is Table 3's rule: sort the element fronts by lowest node
// id, join adjacent pairs round after round, carry an odd last front.  Fronts are numbered in
// post-order, mesh after mesh.
// Pivots (Table 2, Sec. 3.2): a node is eliminated by the first front that holds every element
// touching it -- the lowest common ancestor of those elements' leaves.
// Index list of a front: its pivots ascending, then its contribution block (the children's
// contribution blocks, or a leaf's element nodes, minus the pivots) ascending.
// Foata class (Sec. 3.3): a front depends only on its children, so its class is its height.
#include "plan.hpp"

#include <algorithm>
#include <cstring>
#include <numeric>

namespace mf {

namespace {

struct MeshTree {
  std::vector<int32_t> left, right, elem;   // local ids
  std::vector<int32_t> lo;                  // post-order: subtree of f is [lo[f], f]
};

// Recursive bisection over elems[b, e); returns the post-order id of the subtree root.
int32_t bisect(const int32_t *ijk, int dim, int32_t *elems, int64_t b, int64_t e, MeshTree &t) {
  if (e - b == 1) {
    int32_t id = (int32_t)t.left.size();
    t.left.push_back(-1);
    t.right.push_back(-1);
    t.elem.push_back(elems[b]);
    t.lo.push_back(id);
    return id;
  }
  int32_t mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, mx[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  for (int64_t i = b; i < e; ++i)
    for (int d = 0; d < dim; ++d) {
      int32_t c = ijk[(int64_t)elems[i] * dim + d];
      mn[d] = std::min(mn[d], c);
      mx[d] = std::max(mx[d], c);
    }
  int axis = 0;
  int64_t best = -1;
  for (int d = 0; d < dim; ++d) {
    int64_t len = (int64_t)mx[d] - mn[d] + 1;
    if (len > best) { best = len; axis = d; }
  }
  const int64_t cut = (int64_t)mn[axis] + best / 2;
  int32_t *mid = std::stable_partition(elems + b, elems + e, [&](int32_t el) {
    return (int64_t)ijk[(int64_t)el * dim + axis] < cut;
  });
  const int64_t m = mid - elems;
  const int32_t first = (int32_t)t.left.size();
  int32_t l = bisect(ijk, dim, elems, b, m, t);
  int32_t r = bisect(ijk, dim, elems, m, e, t);
  int32_t id = (int32_t)t.left.size();
  t.left.push_back(l);
  t.right.push_back(r);
  t.elem.push_back(-1);
  t.lo.push_back(first);
  return id;
}

// Table 3 literally: the element fronts sorted by their lowest node id (ties: element id) are
// joined in adjacent pairs, round after round, an odd last front carried to the next round,
// until one front remains.  The tree is then numbered in post-order.
void pairing_tree(const int32_t *conn, int npe, int64_t ne, MeshTree &t) {
  std::vector<int64_t> key(ne);
  for (int64_t e = 0; e < ne; ++e) {
    int32_t lo = INT32_MAX;
    for (int a = 0; a < npe; ++a) lo = std::min(lo, conn[e * npe + a]);
    key[e] = ((int64_t)lo << 32) | (int64_t)e;
  }
  std::vector<int32_t> order(ne);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  std::vector<int32_t> L, R, E, items, next;
  for (int32_t e : order) {
    items.push_back((int32_t)L.size());
    L.push_back(-1);
    R.push_back(-1);
    E.push_back(e);
  }
  while (items.size() > 1) {
    next.clear();
    for (size_t i = 0; i + 1 < items.size(); i += 2) {
      next.push_back((int32_t)L.size());
      L.push_back(items[i]);
      R.push_back(items[i + 1]);
      E.push_back(-1);
    }
    if (items.size() % 2 == 1) next.push_back(items.back());
    items.swap(next);
  }
  // post-order renumbering
  std::vector<int32_t> post(L.size(), -1), lo_of(L.size(), -1);
  std::vector<std::pair<int32_t, int>> st;
  st.push_back({items[0], 0});
  t.left.clear();
  t.right.clear();
  t.elem.clear();
  t.lo.clear();
  while (!st.empty()) {
    auto &[v, state] = st.back();
    if (L[v] >= 0 && state == 0) {
      state = 1;
      st.push_back({L[v], 0});
      continue;
    }
    if (L[v] >= 0 && state == 1) {
      state = 2;
      st.push_back({R[v], 0});
      continue;
    }
    const int32_t id = (int32_t)t.left.size();
    post[v] = id;
    if (L[v] >= 0) {
      t.left.push_back(post[L[v]]);
      t.right.push_back(post[R[v]]);
      t.elem.push_back(-1);
      t.lo.push_back(lo_of[L[v]]);
      lo_of[v] = lo_of[L[v]];
    } else {
      t.left.push_back(-1);
      t.right.push_back(-1);
      t.elem.push_back(E[v]);
      t.lo.push_back(id);
      lo_of[v] = id;
    }
    st.pop_back();
  }
}

}  // namespace

std::string analyse(int32_t n_mesh, const int32_t *dims, const int32_t *npes,
                    const int64_t *n_nodes, const int64_t *n_elems,
                    const int32_t *const *conns, const int32_t *const *ijks, HostPlan &P) {
  if (n_mesh < 1) return "n_mesh must be >= 1";
  P = HostPlan();
  P.n_mesh = n_mesh;
  P.dim = dims[0];
  P.npe = npes[0];
  for (int32_t mi = 0; mi < n_mesh; ++mi) {
    if (dims[mi] != 2 && dims[mi] != 3) return "mesh " + std::to_string(mi) + ": dim must be 2 or 3";
    if (dims[mi] != P.dim) return "all meshes of a batch must have the same dim";
    {
      // Q_p Lagrange elements, p = 1..3: (p+1)^dim nodes per element
      bool ok = false;
      for (int q = 2; q <= 4; ++q) ok |= npes[mi] == (dims[mi] == 2 ? q * q : q * q * q);
      if (!ok) return "mesh " + std::to_string(mi) + ": npe must be (p+1)^dim with p in 1..3";
    }
    if (npes[mi] != P.npe) return "all meshes of a batch must have the same npe";
    if (n_elems[mi] < 1 || n_nodes[mi] < 1) return "mesh " + std::to_string(mi) + ": empty";
    if (!conns[mi]) return "mesh " + std::to_string(mi) + ": null conn";
    if (n_elems[mi] > INT32_MAX / 4 || n_nodes[mi] > INT32_MAX / 4)
      return "mesh " + std::to_string(mi) + ": too large";
    P.n += n_nodes[mi];
    P.n_elem += n_elems[mi];
  }
  if (P.n > INT32_MAX / 2 || P.n_elem > INT32_MAX / 4) return "batch too large for 32-bit ids";
  const int dim = P.dim, npe = P.npe;
  P.conn.resize((size_t)P.n_elem * npe);
  P.F = 2 * P.n_elem - n_mesh;
  const int64_t F = P.F;
  P.parent.assign(F, -1);
  P.level.assign(F, 0);
  P.npiv.assign(F, 0);
  P.width.assign(F, 0);
  P.leaf_elem.assign(F, -1);
  P.front_ptr.assign(F + 1, 0);
  P.desc.resize(F);
  P.front_idx.clear();
  P.inv_l.clear();
  P.inv_r.clear();

  int64_t node_off = 0, elem_off = 0, front_off = 0;
  std::vector<int32_t> owner, cnt, pivs, pos_l, pos_r;
  P.mesh_front_ptr.assign(1, 0);
  P.mesh_node_ptr.assign(1, 0);
  for (int32_t mi = 0; mi < n_mesh; ++mi) {
    const int64_t nn = n_nodes[mi], ne = n_elems[mi];
    const int32_t *conn = conns[mi];
    const int32_t *ijk = ijks[mi];
    // validation: node ids in range, distinct within an element, every node used, ijk unique
    std::vector<uint8_t> used(nn, 0);
    for (int64_t e = 0; e < ne; ++e) {
      for (int a = 0; a < npe; ++a) {
        int32_t v = conn[e * npe + a];
        if (v < 0 || v >= nn)
          return "mesh " + std::to_string(mi) + ": node id out of range in element " + std::to_string(e);
        for (int b = 0; b < a; ++b)
          if (conn[e * npe + b] == v)
            return "mesh " + std::to_string(mi) + ": repeated node in element " + std::to_string(e);
        used[v] = 1;
        P.conn[(elem_off + e) * npe + a] = (int32_t)(v + node_off);
      }
    }
    for (int64_t v = 0; v < nn; ++v)
      if (!used[v]) return "mesh " + std::to_string(mi) + ": node " + std::to_string(v) + " is not used";
    if (ijk) {
      std::vector<int32_t> ord(ne);
      std::iota(ord.begin(), ord.end(), 0);
      std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        return std::lexicographical_compare(ijk + (int64_t)a * dim, ijk + (int64_t)a * dim + dim,
                                            ijk + (int64_t)b * dim, ijk + (int64_t)b * dim + dim);
      });
      for (int64_t i = 1; i < ne; ++i)
        if (std::equal(ijk + (int64_t)ord[i] * dim, ijk + (int64_t)ord[i] * dim + dim,
                       ijk + (int64_t)ord[i - 1] * dim))
          return "mesh " + std::to_string(mi) + ": duplicate elem_ijk";
    }
    // tree
    MeshTree T;
    T.left.reserve(2 * ne);
    if (ijk) {
      std::vector<int32_t> elems(ne);
      std::iota(elems.begin(), elems.end(), 0);
      bisect(ijk, dim, elems.data(), 0, ne, T);
    } else {
      pairing_tree(conn, npe, ne, T);
    }
    const int64_t Fm = (int64_t)T.left.size();
    std::vector<int32_t> par(Fm, -1), leaf_of(ne);
    for (int64_t f = 0; f < Fm; ++f) {
      if (T.left[f] >= 0) { par[T.left[f]] = (int32_t)f; par[T.right[f]] = (int32_t)f; }
      else leaf_of[T.elem[f]] = (int32_t)f;
    }
    // owner = lowest common ancestor of the leaves of the node's elements
    owner.assign(nn, -1);
    for (int64_t e = 0; e < ne; ++e) {
      const int32_t lf = leaf_of[e];
      for (int a = 0; a < npe; ++a) {
        const int32_t v = conn[e * npe + a];
        int32_t o = owner[v];
        if (o < 0) { owner[v] = lf; continue; }
        // climb from o until its post-order interval [lo, o] contains lf
        while (!(T.lo[o] <= lf && lf <= o)) o = par[o];
        owner[v] = o;
      }
    }
    // pivots per front (counting sort keeps node ids ascending)
    cnt.assign(Fm + 1, 0);
    for (int64_t v = 0; v < nn; ++v) cnt[owner[v] + 1]++;
    for (int64_t f = 0; f < Fm; ++f) cnt[f + 1] += cnt[f];
    pivs.assign(nn, 0);
    {
      std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
      for (int64_t v = 0; v < nn; ++v) pivs[fill[owner[v]]++] = (int32_t)v;
    }
    // index lists in post-order (children before parents), extend-add maps
    std::vector<int64_t> lptr(Fm + 1, 0);
    std::vector<int32_t> lidx;          // local index lists of this mesh
    lidx.reserve(8 * Fm);
    std::vector<int32_t> kk(Fm), lvl(Fm, 0);
    std::vector<int32_t> cb;
    for (int64_t f = 0; f < Fm; ++f) {
      const int32_t k = cnt[f + 1] - cnt[f];
      kk[f] = k;
      cb.clear();
      if (T.left[f] < 0) {
        const int32_t e = T.elem[f];
        for (int a = 0; a < npe; ++a) {
          int32_t v = conn[(int64_t)e * npe + a];
          if (owner[v] != f) cb.push_back(v);
        }
        std::sort(cb.begin(), cb.end());
      } else {
        const int32_t l = T.left[f], r = T.right[f];
        lvl[f] = 1 + std::max(lvl[l], lvl[r]);
        const int32_t *a0 = lidx.data() + lptr[l] + kk[l], *a1 = lidx.data() + lptr[l + 1];
        const int32_t *b0 = lidx.data() + lptr[r] + kk[r], *b1 = lidx.data() + lptr[r + 1];
        while (a0 < a1 || b0 < b1) {   // sorted union
          int32_t v;
          if (b0 == b1 || (a0 < a1 && *a0 < *b0)) v = *a0++;
          else if (a0 == a1 || *b0 < *a0) v = *b0++;
          else { v = *a0++; ++b0; }
          if (owner[v] != f) cb.push_back(v);
        }
      }
      lptr[f] = (int64_t)lidx.size();
      for (int32_t i = cnt[f]; i < cnt[f + 1]; ++i) lidx.push_back(pivs[i]);
      lidx.insert(lidx.end(), cb.begin(), cb.end());
      lptr[f + 1] = (int64_t)lidx.size();
    }
    // write this mesh into the global plan
    for (int64_t f = 0; f < Fm; ++f) {
      const int64_t g = front_off + f;
      const int32_t m = (int32_t)(lptr[f + 1] - lptr[f]);
      const int32_t k = kk[f];
      P.parent[g] = par[f] < 0 ? -1 : (int32_t)(par[f] + front_off);
      P.level[g] = lvl[f];
      P.npiv[g] = k;
      P.width[g] = m;
      P.leaf_elem[g] = T.elem[f] < 0 ? -1 : (int64_t)T.elem[f] + elem_off;
      P.front_ptr[g + 1] = P.front_ptr[g] + m;
      FrontDesc &d = P.desc[g];
      d.m = m;
      d.k = k;
      d.left = T.left[f] < 0 ? -1 : (int32_t)(T.left[f] + front_off);
      d.right = T.right[f] < 0 ? -1 : (int32_t)(T.right[f] + front_off);
      d.elem = T.elem[f] < 0 ? -1 : (int32_t)(T.elem[f] + elem_off);
      d.level = lvl[f];
      const int32_t *lst = lidx.data() + lptr[f];
      for (int32_t i = 0; i < m; ++i) P.front_idx.push_back((int32_t)(lst[i] + node_off));
      if (T.left[f] < 0) {
        const int32_t e = T.elem[f];
        for (int32_t i = 0; i < m; ++i) {
          int32_t a = 0;
          while (conn[(int64_t)e * npe + a] != lst[i]) ++a;
          P.inv_l.push_back(a);
          P.inv_r.push_back(-1);
        }
      } else {
        const int32_t c2[2] = {T.left[f], T.right[f]};
        for (int32_t i = 0; i < m; ++i) {
          int32_t pos[2];
          for (int s = 0; s < 2; ++s) {
            const int32_t c = c2[s];
            if (T.left[c] < 0 && kk[c] == 0) {
              // pass-through leaf (no pivots): its contribution block is its element matrix, so
              // the map points straight at the element's local node
              pos[s] = -1;
              for (int a = 0; a < npe; ++a)
                if (conn[(int64_t)T.elem[c] * npe + a] == lst[i]) pos[s] = a;
              continue;
            }
            const int32_t *b0 = lidx.data() + lptr[c] + kk[c], *b1 = lidx.data() + lptr[c + 1];
            const int32_t *it = std::lower_bound(b0, b1, lst[i]);
            pos[s] = (it != b1 && *it == lst[i]) ? (int32_t)(it - b0) : -1;
          }
          P.inv_l.push_back(pos[0]);
          P.inv_r.push_back(pos[1]);
        }
      }
    }
    node_off += nn;
    elem_off += ne;
    front_off += Fm;
    P.mesh_front_ptr.push_back(front_off);
    P.mesh_node_ptr.push_back(node_off);
  }
  // offsets, counts
  int64_t store = 0, cbrow = 0;
  P.height = 0;
  for (int64_t f = 0; f < F; ++f) {
    FrontDesc &d = P.desc[f];
    d.idx = P.front_ptr[f];
    d.store = store;
    d.cbrow = cbrow;
    store += (int64_t)d.m * d.m;
    cbrow += d.m - d.k;
    P.sum_mk += (int64_t)d.m * d.k;
    P.height = std::max(P.height, d.level);
    P.max_m = std::max(P.max_m, d.m);
    P.max_k = std::max(P.max_k, d.k);
    for (int32_t p = 0; p < d.k; ++p) {
      const double r = (double)(d.m - p);
      P.factor_flops += (r - 1) + 2 * (r - 1) * (r - 1);
      P.solve_flops += 1 + 4 * (r - 1);
    }
    P.sum_cb2 += (double)(d.m - d.k) * (d.m - d.k);
  }
  P.store_doubles = store;
  P.sum_c = cbrow;
  build_schedule(P, std::vector<Tuning>(P.height + 1, Tuning()));
  return "";
}

void build_schedule(HostPlan &P, const std::vector<Tuning> &tl) {
  P.levels.assign(P.height + 1, LevelSchedule());
  for (int64_t f = 0; f < P.F; ++f) {
    const FrontDesc &d = P.desc[f];
    if (d.elem >= 0 && d.k == 0) continue;   // pass-through leaf: read directly by its parent
    LevelSchedule &L = P.levels[d.level];
    const Tuning &t = tl[d.level];
    L.max_m = std::max(L.max_m, d.m);
    L.max_k = std::max(L.max_k, d.k);
    if (d.m <= std::min(t.tiny_max_m, t.small_max_m)) {
      L.tiny.push_back((int32_t)f);
      L.tiny_max_m = std::max(L.tiny_max_m, d.m);
    } else if (d.m <= t.small_max_m) {
      L.small.push_back((int32_t)f);
      L.small_max_m = std::max(L.small_max_m, d.m);
    } else {
      L.large.push_back((int32_t)f);
      L.large_max_m = std::max(L.large_max_m, d.m);
    }
  }
  // a class with at most as many tiny fronts as small ones runs them on the small route too:
  // one launch for the class instead of two in sequence (the two routes' arithmetic is the
  // same elimination; a few tiny fronts are not worth a launch of their own)
  for (auto &L : P.levels) {
    if (L.small.empty() || L.tiny.empty() || L.tiny.size() > L.small.size()) continue;
    L.small.insert(L.small.begin(), L.tiny.begin(), L.tiny.end());
    L.tiny.clear();
    L.tiny_max_m = 0;
  }
  // the solve's list of a class: the tiny fronts first (their wave records are then a prefix
  // of the class's records), then the rest; fronts of a class are independent
  for (auto &L : P.levels) {
    L.all.clear();
    L.all.insert(L.all.end(), L.tiny.begin(), L.tiny.end());
    L.all.insert(L.all.end(), L.small.begin(), L.small.end());
    L.all.insert(L.all.end(), L.large.begin(), L.large.end());
  }
  // the persistent class launch runs every tiled front panel by panel, 32 pivots at a time
  int32_t T = 64;
  auto add_tiles = [&](std::vector<GemmTask> &out, int32_t f, int32_t i0, int32_t i1, int32_t j0,
                       int32_t j1, int32_t q0, int32_t q1) {
    if (i0 >= i1 || j0 >= j1 || q0 >= q1) return;
    for (int32_t i = i0; i < i1; i += T)
      for (int32_t j = j0; j < j1; j += T) {
        GemmTask g;
        g.front = f;
        g.store = P.desc[f].store;
        g.ld = P.desc[f].m;
        g.i0 = i;
        g.i1 = std::min(i + T, i1);
        g.j0 = j;
        g.j1 = std::min(j + T, j1);
        g.q0 = q0;
        g.q1 = q1;
        out.push_back(g);
      }
  };
  for (size_t l = 0; l < P.levels.size(); ++l) {
    LevelSchedule &L = P.levels[l];
    const Tuning &t = tl[l];
    const int32_t nb = t.persistent ? 32 : t.nb;
    const int32_t fused_lim = t.persistent ? 0 : t.fused_max_m;
    T = t.tile;
    int32_t max_steps = 0;
    for (int32_t f : L.large) {
      const FrontDesc &d = P.desc[f];
      if (d.m <= fused_lim) {
        if (d.k > 0) {
          L.fused.push_back(f);
          L.fused_max_m = std::max(L.fused_max_m, d.m);
        }
      } else {
        max_steps = std::max(max_steps, (d.k + nb - 1) / nb);
      }
    }
    L.steps.assign(max_steps, PanelStep());
    L.lookahead = !t.persistent && nb == 32;
    for (int32_t f : L.large) {
      const FrontDesc &d = P.desc[f];
      add_tiles(L.schur, f, d.k, d.m, d.k, d.m, 0, d.k);
      if (d.m <= fused_lim) continue;
      for (int32_t s = 0; s * nb < d.k; ++s) {
        const int32_t p0 = s * nb, pe = std::min(p0 + nb, d.k);
        PanelStep &S = L.steps[s];
        S.fronts.push_back(f);
        S.p0.push_back(p0);
        // columns, then rows from the next multiple of 64 (see k_panel_trsm)
        S.trsm_items = std::max<int64_t>(S.trsm_items, (int64_t)((d.m - pe + 63) & ~63) + (d.m - pe));
        // fully-summed region still to update by this panel: rows [pe,k) x cols [pe,m) and rows
        // [k,m) x cols [pe,k); in the look-ahead form the next step's launch does it beyond the
        // next panel (its own rows and columns the next panel updates itself)
        if (L.lookahead) {
          if (pe < d.k) {
            PanelStep &N = L.steps[s + 1];
            const int32_t pn = std::min(pe + nb, d.k);
            add_tiles(N.prev_update, f, pn, d.k, pn, d.k, p0, pe);
            add_tiles(N.prev_update, f, pn, d.k, d.k, d.m, p0, pe);
            add_tiles(N.prev_update, f, d.k, d.m, pn, d.k, p0, pe);
          }
        } else {
          add_tiles(S.update, f, pe, d.k, pe, d.k, p0, pe);
          add_tiles(S.update, f, pe, d.k, d.k, d.m, p0, pe);
          add_tiles(S.update, f, d.k, d.m, pe, d.k, p0, pe);
        }
      }
    }
  }
}

}  // namespace mf
