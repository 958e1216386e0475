"""Active-set logic of Algorithms 1 and 2 with Python sets (oracle; test
infrastructure only).

Definitions (Section 4.3):

* V_A: active cells; V_B: the outermost layer of V_A, read here as the
  active cells with at least one neighbour outside V_A;
* V_nbr^{i,m}: the cells within m layers of i.  Fig. 2, which draws it, is
  not available; it is read as all cells at graph distance <= m from i over
  the connection graph (matrix, fracture and non-neighbour connections),
  i included;
* a cell's update is non-negligible when |dp_i| >= eps (the cutoff is a
  pressure quantity in Section 5);
* the outer layer dB of a set (Section 4.4, Step 1): the cells outside the
  set adjacent to it;
* the residual-based estimate that Sections 1 and 4.2 attribute to Lu and
  Beckner: the unconverged cells (error measure at or above a tolerance)
  inflated by a fixed number of neighbour layers, one by default;
* localized fracture cells (Section 5.2.3 keeps fracture cells active and
  notes that localizing them would save more work): fracture cells that
  are not always active join the active set a whole fracture component at
  a time -- a component being the fracture cells connected through
  fracture-fracture connections (intersections included) -- because a
  pressure change crosses such a component within one step while the
  m-layer growth advances m cells per iteration.  Every active set of
  Algorithm 1 is closed under components (frac_closure); with all fracture
  cells always active the closure changes nothing.

Everything here is the plain definition over Python sets; nothing is
vectorized.
"""
from __future__ import annotations


def neighbours(rp, nb, i):
    return nb[rp[i]:rp[i + 1]]


def ball(rp, nb, i, m):
    """V_nbr^{i,m}: breadth-first search to depth m."""
    seen = {int(i)}
    frontier = [int(i)]
    for _ in range(m):
        nxt = []
        for c in frontier:
            for j in neighbours(rp, nb, c):
                j = int(j)
                if j not in seen:
                    seen.add(j)
                    nxt.append(j)
        frontier = nxt
    return seen


def boundary(rp, nb, act):
    """V_B: active cells with a neighbour outside the active set."""
    return {i for i in act
            if any(int(j) not in act for j in neighbours(rp, nb, i))}


def outer_layer(rp, nb, act):
    """dB: cells outside ``act`` adjacent to it."""
    out = set()
    for i in act:
        for j in neighbours(rp, nb, i):
            if int(j) not in act:
                out.add(int(j))
    return out


def fracture_components(rp, nb, is_frac):
    """Connected components of the fracture cells over fracture-fracture
    connections: (comp, members) with comp[i] the component of cell i (-1
    for matrix cells) and members[c] the set of cells of component c."""
    n = len(is_frac)
    comp = [-1] * n
    members = []
    for i in range(n):
        if not is_frac[i] or comp[i] >= 0:
            continue
        c = len(members)
        comp[i] = c
        todo, cells = [i], {i}
        while todo:
            a = todo.pop()
            for j in neighbours(rp, nb, a):
                j = int(j)
                if is_frac[j] and comp[j] < 0:
                    comp[j] = c
                    cells.add(j)
                    todo.append(j)
        members.append(cells)
    return comp, members


def frac_closure(act, comp, members):
    """The set plus every fracture component it touches."""
    out = set(act)
    for c in {comp[i] for i in act if comp[i] >= 0}:
        out |= members[c]
    return out


def initial_active(rp, nb, always_active, m, prev_support=None, fcomp=None):
    """Initial V_A.  First step: the wells / fractures and their m-layer
    neighbourhood (Section 4.3 remark on the initial set); later steps:
    the support of the previous timestep plus the always-active cells
    (Section 5.2.1 takes the last timestep's support).  fcomp: the
    (comp, members) pair of localized fracture cells, or None."""
    aa = {int(i) for i in always_active}
    if prev_support is None:
        out = set()
        for i in aa:
            out |= ball(rp, nb, i, m)
    else:
        out = {int(i) for i in prev_support} | aa
    return frac_closure(out, *fcomp) if fcomp else out


def alg1_update(rp, nb, act, bnd, dp_abs, eps, m, always_active, fcomp=None):
    """One pass of the set logic of Algorithm 1 after a local solve.

    For each boundary cell with a non-negligible update, V_A grows by its
    m-layer neighbourhood ('expand').  If no boundary update is
    non-negligible, V_A becomes the support of the update plus the
    always-active cells ('shrink').  With localized fracture cells (fcomp)
    the new set is closed under fracture components.  Returns (act, bnd,
    is_expand)."""
    new = set(act)
    is_expand = False
    for i in bnd:
        if dp_abs[i] >= eps:
            is_expand = True
            new |= ball(rp, nb, i, m)
    if not is_expand:
        new = {i for i in act if dp_abs[i] >= eps} | {int(i) for i in always_active}
    if fcomp:
        new = frac_closure(new, *fcomp)
    return new, boundary(rp, nb, new), is_expand


def alg2_expand(rp, nb, vt, bnd_k, dp_abs, eps, m):
    """Phase-1 set logic of Algorithm 2 after the local solve on V_A^k.

    Returns (V_A^{k+1}, V_T, V_B^{k+1}, dB^{k+1}, is_expand)."""
    nxt = set()
    vt = set(vt)
    is_expand = False
    for i in bnd_k:
        if dp_abs[i] >= eps:
            is_expand = True
            bl = ball(rp, nb, i, m)
            vt |= bl
            nxt |= bl
    if not is_expand:
        return set(), vt, set(), set(), False
    vb_t = boundary(rp, nb, vt)
    return nxt, vt, vb_t & nxt, outer_layer(rp, nb, nxt), True


def alg2_sub_max(cells, outer, last_dp):
    """Phase-2 skip test of Algorithm 2 (Section 4.4, Step 2): the largest
    latest update over subdomain V_A^k and its outer layer dB^k (0 for two
    empty lists).  The subdomain is solved when this is at least eps."""
    vals = [float(last_dp[int(i)]) for i in cells] + [float(last_dp[int(i)]) for i in outer]
    return max(vals) if vals else 0.0


def alg2_owner(subdomains, n):
    """The additive form of Algorithm 2's phase 2 combines overlapping
    updates by ownership: cell i takes the update of the first subdomain
    (in build order) that contains it; -1 for cells in none."""
    owner = [-1] * n
    for k, cells in enumerate(subdomains):
        for i in cells:
            if owner[int(i)] < 0:
                owner[int(i)] = k
    return owner


def resid_active(rp, nb, err, tol, layers):
    """Residual-based active set (Sections 1 and 4.2, the estimator of Lu
    and Beckner): every cell with err_i >= tol, inflated by its
    ``layers``-layer neighbourhood."""
    out = set()
    for i in range(len(err)):
        if err[i] >= tol:
            out |= ball(rp, nb, i, layers)
    return out
