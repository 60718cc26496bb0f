// Host set-up of the patch form of the operator passes (patch.hip).
//
// Elements are grouped into patches of at most P elements (one work-group
// each) by greedy graph growing over the element graph of the local-to-global
// map (two elements are neighbours when they share a DOF): a patch starts at
// the most enclosed unassigned element (the most DOF incidences shared with
// elements already assigned; the lowest-numbered unassigned one when none is
// enclosed) and repeatedly takes the unassigned neighbour with the most DOF
// copies already in the patch, which keeps patches compact, so that most of
// their DOFs have every broken copy inside.  Growth stops at P - P/8
// elements; afterwards a patch of fewer than a quarter of that joins the
// neighbouring patch it shares the most copies with, where elements and DOFs
// fit.  The library then numbers elements patch by patch (all element-indexed
// data follow that internal order).
//
// For each patch the plan lists its DOFs (those whose copies all lie in the
// patch first, then the shared ones, each group in increasing DOF order) and,
// for each broken copy (K, l), a code = j | rank << lbits: j the copy's DOF in
// the patch list and rank its position among that DOF's copies of the patch,
// counted in element order.  The element pass adds copies of rank 0, 1, ...
// in turn, so each DOF's copies are summed in one fixed order without float
// atomics.  A shared DOF gets one partial sum per patch; the partials are
// summed in patch order by a second pass over the shared DOFs.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "patch.h"

namespace bras {

namespace {

// Max-gain bucket queue with lazy deletion; within a bucket the most
// recently pushed entry is taken first (a fixed, data-dependent order).
struct BucketQueue {
  std::vector<std::vector<int32_t>> b;
  int top = -1;
  void push(int g, int32_t k) {
    if (g >= (int)b.size()) b.resize(g + 1);
    b[g].push_back(k);
    if (g > top) top = g;
  }
  void clear() {
    for (auto& v : b) v.clear();
    top = -1;
  }
};

}  // namespace

int build_patch_plan(int64_t n, int64_t E, int nl, const int32_t* l2g, const int32_t* mult, int P, int Dmax,
                     PatchPlan* plan) {
  if (P < 1) return 1;
  // 16-bit codes: rank bits for the largest multiplicity, the rest for j
  int maxmult = 1;
  for (int64_t i = 0; i < n; ++i) maxmult = std::max(maxmult, (int)mult[i]);
  int rbits = 0;
  while ((1 << rbits) < maxmult) ++rbits;
  if (rbits > 10) return 1;
  Dmax = std::min(Dmax, 1 << (16 - rbits));
  if (Dmax < nl) return 1;
  // DOF -> elements (CSR)
  std::vector<int64_t> drp(n + 1, 0);
  for (int64_t q = 0; q < E * nl; ++q) ++drp[l2g[q] + 1];
  for (int64_t i = 0; i < n; ++i) drp[i + 1] += drp[i];
  std::vector<int32_t> del(E * nl);
  {
    std::vector<int64_t> fill(drp.begin(), drp.end() - 1);
    for (int64_t K = 0; K < E; ++K)
      for (int l = 0; l < nl; ++l) del[fill[l2g[K * nl + l]]++] = (int32_t)K;
  }
  std::vector<int32_t> part(E, -1);
  std::vector<int32_t> gain(E, 0);
  std::vector<int32_t> anc(E, 0);     // DOF incidences shared with already assigned elements
  std::vector<int32_t> stamp(n, -1);
  std::vector<int32_t> touched;
  BucketQueue bq;
  BucketQueue seeds;                  // unassigned elements by anc: a new patch starts at the most
                                      // enclosed one, so that no small pockets are left behind
  plan->perm.clear();
  plan->perm.reserve(E);
  plan->pe.assign(1, 0);
  int64_t next = 0;
  int32_t np = 0;
  // patches grow to Pg < P elements; the room left takes in the small
  // pockets greedy growth leaves between patches (merge step below)
  const int Pg = P >= 16 ? P - P / 8 : P;
  while (true) {
    int32_t seed = -1;
    while (seeds.top > 0 && seed < 0) {
      auto& v = seeds.b[seeds.top];
      if (v.empty()) {
        --seeds.top;
        continue;
      }
      const int32_t k = v.back();
      v.pop_back();
      if (part[k] < 0 && anc[k] == seeds.top) seed = k;
    }
    if (seed < 0) {
      while (next < E && part[next] >= 0) ++next;
      if (next >= E) break;
      seed = (int32_t)next;
    }
    bq.clear();
    touched.clear();
    bq.push(0, seed);
    int cnt = 0, ndof = 0;
    while (cnt < Pg) {
      int32_t K = -1;
      while (bq.top >= 0 && K < 0) {
        auto& v = bq.b[bq.top];
        if (v.empty()) {
          --bq.top;
          continue;
        }
        const int32_t k = v.back();
        v.pop_back();
        if (part[k] < 0 && gain[k] == bq.top) K = k;
      }
      if (K < 0) break;   // frontier exhausted: the patch ends small
      int add = 0;
      for (int l = 0; l < nl; ++l) add += stamp[l2g[(int64_t)K * nl + l]] != np;
      if (ndof + add > Dmax) break;
      part[K] = np;
      plan->perm.push_back(K);
      ++cnt;
      ndof += add;
      for (int l = 0; l < nl; ++l) {
        const int32_t g = l2g[(int64_t)K * nl + l];
        stamp[g] = np;
        for (int64_t a = drp[g]; a < drp[g + 1]; ++a) {
          const int32_t K2 = del[a];
          if (part[K2] >= 0) continue;
          if (gain[K2] == 0) touched.push_back(K2);
          ++gain[K2];
          bq.push(gain[K2], K2);
          ++anc[K2];
        }
      }
    }
    for (int32_t k : touched) {
      gain[k] = 0;
      if (part[k] < 0) seeds.push(anc[k], k);
    }
    ++np;
  }
  // merge: a patch of fewer than Pg / 4 elements joins the neighbouring patch
  // it shares the most DOF copies with, when that one has room for its
  // elements and DOFs
  {
    std::vector<int32_t> ecount(np, 0), dcount(np, 0);
    for (int64_t K = 0; K < E; ++K) ++ecount[part[K]];
    std::vector<int32_t> dstamp(n, -1);
    for (int64_t K = 0; K < E; ++K)
      for (int l = 0; l < nl; ++l) {
        const int32_t g = l2g[K * nl + l];
        if (dstamp[g] != part[K]) {
          // a DOF is counted once per patch: its elements' patches are visited in element order
          bool seen = false;
          for (int64_t a = drp[g]; a < drp[g + 1] && del[a] < K; ++a) seen = seen || part[del[a]] == part[K];
          if (!seen) ++dcount[part[K]];
          dstamp[g] = part[K];
        }
      }
    std::vector<std::vector<int32_t>> members(np);
    for (int32_t K : plan->perm) members[part[K]].push_back(K);   // growth order
    std::vector<int32_t> score(np, 0), cand;
    for (int32_t q = 0; q < np; ++q) {
      if (ecount[q] == 0 || ecount[q] >= Pg / 4) continue;
      cand.clear();
      for (int32_t K : members[q])
        for (int l = 0; l < nl; ++l) {
          const int32_t g = l2g[(int64_t)K * nl + l];
          for (int64_t a = drp[g]; a < drp[g + 1]; ++a) {
            const int32_t t = part[del[a]];
            if (t == q) continue;
            if (score[t] == 0) cand.push_back(t);
            ++score[t];
          }
        }
      int32_t best = -1;
      for (int32_t t : cand) {
        if (ecount[t] + ecount[q] > P) continue;
        if (best < 0 || score[t] > score[best] || (score[t] == score[best] && t < best)) best = t;
      }
      for (int32_t t : cand) score[t] = 0;
      if (best < 0) continue;
      // DOFs the merged patch would hold
      int add = 0;
      for (int32_t K : members[q])
        for (int l = 0; l < nl; ++l) {
          const int32_t g = l2g[(int64_t)K * nl + l];
          bool in_best = false, first = true;
          for (int64_t a = drp[g]; a < drp[g + 1]; ++a) {
            const int32_t t = part[del[a]];
            in_best = in_best || t == best;
            if (t == q && del[a] < K) first = false;
          }
          if (!in_best && first) ++add;
        }
      if (dcount[best] + add > Dmax) continue;
      for (int32_t K : members[q]) {
        part[K] = best;
        members[best].push_back(K);
      }
      members[q].clear();
      ecount[best] += ecount[q];
      ecount[q] = 0;
      dcount[best] += add;
      dcount[q] = 0;
    }
    // patch-major element order, patches in creation order, elements in growth order
    plan->perm.clear();
    for (int32_t q = 0; q < np; ++q) {
      if (members[q].empty()) continue;
      for (int32_t K : members[q]) plan->perm.push_back(K);
      plan->pe.push_back((int32_t)plan->perm.size());
    }
  }
  const int64_t npatch = (int64_t)plan->pe.size() - 1;
  plan->npatch = npatch;
  // per-patch DOF lists: local DOFs (every copy in the patch) first, by DOF;
  // then the shared ones, in the order of the shared-DOF numbering below
  std::vector<int32_t> lj(n, -1);       // DOF -> index in the current patch's first-seen list
  std::vector<int32_t> seen, cnt_in;    // first-seen DOF list and copy counts
  std::vector<int64_t> lloc_off(npatch + 1, 0), lsh_off(npatch + 1, 0);
  std::vector<int32_t> lloc, lsh;       // per patch: local DOFs (sorted), shared DOFs (unsorted)
  std::vector<int32_t> shared_cnt(n, 0);
  for (int64_t p = 0; p < npatch; ++p) {
    const int32_t e0 = plan->pe[p], e1 = plan->pe[p + 1];
    seen.clear();
    cnt_in.clear();
    for (int32_t e = e0; e < e1; ++e) {
      const int64_t K = plan->perm[e];
      for (int l = 0; l < nl; ++l) {
        const int32_t g = l2g[K * nl + l];
        if (lj[g] < 0) {
          lj[g] = (int32_t)seen.size();
          seen.push_back(g);
          cnt_in.push_back(0);
        }
        ++cnt_in[lj[g]];
      }
    }
    const size_t l0 = lloc.size();
    for (size_t k = 0; k < seen.size(); ++k) {
      const int32_t g = seen[k];
      if (cnt_in[k] == mult[g]) {
        lloc.push_back(g);
      } else {
        lsh.push_back(g);
        ++shared_cnt[g];
      }
      lj[g] = -1;
    }
    std::sort(lloc.begin() + l0, lloc.end());
    lloc_off[p + 1] = (int64_t)lloc.size();
    lsh_off[p + 1] = (int64_t)lsh.size();
  }
  // Shared DOFs ordered by the list of patches that hold them, then by DOF:
  // the DOFs of one interface between patches are then consecutive, both in
  // this numbering and in each of those patches' lists, so the second pass
  // reads their partial sums in runs.
  std::vector<int64_t> sp_off(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) sp_off[i + 1] = sp_off[i] + shared_cnt[i];
  std::vector<int32_t> sp_list(sp_off[n]);   // patches of each shared DOF, increasing
  {
    std::vector<int64_t> fill(sp_off.begin(), sp_off.end() - 1);
    for (int64_t p = 0; p < npatch; ++p)
      for (int64_t k = lsh_off[p]; k < lsh_off[p + 1]; ++k) sp_list[fill[lsh[k]]++] = (int32_t)p;
  }
  plan->sdof.clear();
  for (int64_t i = 0; i < n; ++i)
    if (shared_cnt[i] > 0) plan->sdof.push_back((int32_t)i);
  std::sort(plan->sdof.begin(), plan->sdof.end(), [&](int32_t a, int32_t b) {
    const int64_t na = sp_off[a + 1] - sp_off[a], nb = sp_off[b + 1] - sp_off[b];
    for (int64_t k = 0; k < na && k < nb; ++k)
      if (sp_list[sp_off[a] + k] != sp_list[sp_off[b] + k]) return sp_list[sp_off[a] + k] < sp_list[sp_off[b] + k];
    if (na != nb) return na < nb;
    return a < b;
  });
  std::vector<int32_t> sidx(n, -1);
  for (size_t k = 0; k < plan->sdof.size(); ++k) sidx[plan->sdof[k]] = (int32_t)k;
  // final patch lists, copy codes and ranks
  plan->pd.assign(1, 0);
  plan->pnl.assign(npatch, 0);
  plan->pdof.clear();
  plan->sbase.assign(npatch + 1, 0);
  std::vector<uint32_t> jr(E * nl, 0);   // (j, rank) per copy, packed below
  std::vector<int32_t> jof(n, -1), rk;
  int maxd = 0, maxr = 0;
  for (int64_t p = 0; p < npatch; ++p) {
    const int32_t e0 = plan->pe[p], e1 = plan->pe[p + 1], ne = e1 - e0;
    const int64_t d0 = (int64_t)plan->pdof.size();
    for (int64_t k = lloc_off[p]; k < lloc_off[p + 1]; ++k) plan->pdof.push_back(lloc[k]);
    std::sort(lsh.begin() + lsh_off[p], lsh.begin() + lsh_off[p + 1],
              [&](int32_t a, int32_t b) { return sidx[a] < sidx[b]; });
    for (int64_t k = lsh_off[p]; k < lsh_off[p + 1]; ++k) plan->pdof.push_back(lsh[k]);
    const int nd = (int)((int64_t)plan->pdof.size() - d0);
    const int nloc = (int)(lloc_off[p + 1] - lloc_off[p]);
    for (int k = 0; k < nd; ++k) jof[plan->pdof[d0 + k]] = k;
    plan->pnl[p] = nloc;
    plan->pd.push_back((int32_t)plan->pdof.size());
    plan->sbase[p + 1] = plan->sbase[p] + (nd - nloc);
    maxd = std::max(maxd, nd);
    // ranks in element order
    rk.assign(nd, 0);
    for (int32_t e = e0; e < e1; ++e) {
      const int64_t K = plan->perm[e];
      for (int l = 0; l < nl; ++l) {
        const int32_t j = jof[l2g[K * nl + l]];
        const int32_t r = rk[j]++;
        maxr = std::max(maxr, r);
        // j and r packed once lbits is known: keep (j, r) for now
        jr[(int64_t)e0 * nl + (int64_t)l * ne + (e - e0)] = (uint32_t)j | ((uint32_t)r << 16);
      }
    }
    for (int k = 0; k < nd; ++k) jof[plan->pdof[d0 + k]] = -1;
  }
  // code packing: lbits for j, the rank above (maxd <= Dmax <= 2^(16 - rbits), maxr < maxmult <= 2^rbits)
  int lbits = 1;
  while ((1 << lbits) < maxd) ++lbits;
  if (lbits + rbits > 16) return 1;
  plan->lbits = lbits;
  plan->rbits = rbits;
  plan->maxrank = maxr;
  plan->maxdofs = maxd;
  plan->code.resize(E * nl);
  for (int64_t q = 0; q < E * nl; ++q) {
    const uint32_t cd = (jr[q] & 0xFFFFu) | ((jr[q] >> 16) << lbits);
    if (cd == 0xFFFFu) return 1;   // reserved by the matrix-core pass for "no output"
    plan->code[q] = (uint16_t)cd;
  }
  // second pass: shared DOF s has partials spos[srp[s] .. srp[s+1]), one per
  // patch that holds it, in patch order (patches write theirs patch-major)
  const int64_t ns = (int64_t)plan->sdof.size();
  plan->srp.assign(ns + 1, 0);
  for (int64_t k = 0; k < ns; ++k) plan->srp[k + 1] = plan->srp[k] + shared_cnt[plan->sdof[k]];
  plan->spos.assign(plan->srp[ns], 0);
  {
    std::vector<int32_t> fill(plan->srp.begin(), plan->srp.end() - 1);
    for (int64_t p = 0; p < npatch; ++p) {
      const int32_t d0 = plan->pd[p], d1 = plan->pd[p + 1], nloc = plan->pnl[p];
      for (int32_t j = d0 + nloc; j < d1; ++j) {
        const int32_t s = sidx[plan->pdof[j]];
        plan->spos[fill[s]++] = plan->sbase[p] + (j - d0 - nloc);
      }
    }
  }
  // internal numbering: local DOFs patch by patch, then the shared DOFs
  int64_t nloc_total = 0;
  for (int64_t p = 0; p < npatch; ++p) nloc_total += plan->pnl[p];
  plan->nloc_total = nloc_total;
  plan->ip2g.assign(n, -1);
  plan->pidx.assign(plan->pdof.size(), 0);
  std::vector<int32_t> g2ip(n, -1);
  for (size_t k = 0; k < plan->sdof.size(); ++k) {
    plan->ip2g[nloc_total + (int64_t)k] = plan->sdof[k];
    g2ip[plan->sdof[k]] = (int32_t)(nloc_total + (int64_t)k);
  }
  int64_t lb = 0;
  for (int64_t p = 0; p < npatch; ++p) {
    const int32_t d0 = plan->pd[p], d1 = plan->pd[p + 1], nloc = plan->pnl[p];
    for (int32_t j = d0; j < d1; ++j) {
      const int32_t g = plan->pdof[j];
      if (j - d0 < nloc) {
        // the patch passes rely on this: local DOF j of patch p is pd[p] - sbase[p] + j
        if (lb != (int64_t)d0 - plan->sbase[p] + (j - d0)) return 1;
        plan->ip2g[lb] = g;
        plan->pidx[j] = (int32_t)lb++;
      } else {
        plan->pidx[j] = g2ip[g];
      }
    }
  }
  for (int64_t i = 0; i < n; ++i)
    if (plan->ip2g[i] < 0) return 1;   // every DOF has a copy, so this cannot happen
  return 0;
}

}  // namespace bras
