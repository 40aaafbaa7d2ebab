"""Exact optimal-transport solvers used to pin the oracle (tests only).

None of these share code with the oracle or with the GPU path; each is a
textbook method that reaches the exact optimum of the LP (eq. ot of the paper)
on the inputs it accepts:

* :func:`transport_simplex`  -- network simplex specialised to the transportation
  problem (north-west-corner start, u/v potentials on the basis tree, Bland's rule),
  for tiny instances;
* :func:`assignment_brute_force` -- uniform marginals f = g = 1/n: by Birkhoff-von
  Neumann an optimal plan is a permutation matrix / n, so OPT is the best of n!
  permutations;
* :func:`w1_line_closed_form` -- 1-D W1 on a common uniform grid: spacing times the
  L1 distance between the two CDFs;
* :func:`monotone_coupling` -- 1-D convex costs: the north-west-corner coupling of
  the sorted supports is optimal.
"""
import itertools

import numpy as np


def transport_simplex(C, f, g, max_pivots=100000, eps=1e-14):
    """Return (OPT, X) of min <C,X> s.t. X1=f, X^T1=g, X>=0 (requires sum f = sum g)."""
    C = np.asarray(C, dtype=np.float64)
    m, n = C.shape
    a = np.array(f, dtype=np.float64)
    b = np.array(g, dtype=np.float64)
    b[-1] += a.sum() - b.sum()           # exact balance for the start basis
    X = np.zeros((m, n))
    basis = []
    i = j = 0
    while True:                           # north-west corner: m+n-1 basic cells
        x = min(a[i], b[j])
        X[i, j] = x
        basis.append((i, j))
        a[i] -= x
        b[j] -= x
        if i == m - 1 and j == n - 1:
            break
        if (a[i] <= 0.0 and i < m - 1) or j == n - 1:
            i += 1
        else:
            j += 1
    basis = set(basis)
    for _ in range(max_pivots):
        # potentials u_i + v_j = C_ij on the basis tree (rows 0..m-1, columns m..m+n-1)
        adj = {k: [] for k in range(m + n)}
        for (r, c) in basis:
            adj[r].append(m + c)
            adj[m + c].append(r)
        pot = {0: 0.0}
        stack = [0]
        while stack:
            node = stack.pop()
            for nb in adj[node]:
                if nb in pot:
                    continue
                if node < m:   # node is row i, nb is column j: v_j = C_ij - u_i
                    pot[nb] = C[node, nb - m] - pot[node]
                else:          # node is column j, nb is row i: u_i = C_ij - v_j
                    pot[nb] = C[nb, node - m] - pot[node]
                stack.append(nb)
        u = np.array([pot[r] for r in range(m)])
        v = np.array([pot[m + c] for c in range(n)])
        red = C - u[:, None] - v[None, :]
        scale = max(1.0, np.abs(C).max())
        enter = None
        for r in range(m):                 # Bland: first improving cell
            for c in range(n):
                if (r, c) not in basis and red[r, c] < -eps * scale:
                    enter = (r, c)
                    break
            if enter:
                break
        if enter is None:
            return float((C * X).sum()), X
        # path in the tree from column enter_c to row enter_r
        r0, c0 = enter
        start, goal = m + c0, r0
        prev = {start: None}
        queue = [start]
        while queue:
            node = queue.pop(0)
            if node == goal:
                break
            for nb in adj[node]:
                if nb not in prev:
                    prev[nb] = node
                    queue.append(nb)
        path_nodes = []
        node = goal
        while node is not None:
            path_nodes.append(node)
            node = prev[node]
        path_nodes.reverse()               # column c0 ... row r0
        cells = []
        for k in range(len(path_nodes) - 1):
            s, t = path_nodes[k], path_nodes[k + 1]
            cells.append((t, s - m) if s >= m else (s, t - m))
        # the entering cell gains theta; cells along the path alternate -, +, -, ...
        minus = cells[0::2]
        plus = cells[1::2]
        theta = min(X[c] for c in minus)
        leave = min((c for c in minus if X[c] == theta))
        for c in minus:
            X[c] -= theta
        for c in plus:
            X[c] += theta
        X[enter] += theta
        basis.remove(leave)
        basis.add(enter)
    raise RuntimeError("transport simplex did not terminate")


def assignment_brute_force(C):
    """Uniform marginals 1/n: OPT = min over permutations of mean C_{i, s(i)}."""
    C = np.asarray(C, dtype=np.float64)
    n = C.shape[0]
    best = np.inf
    rows = np.arange(n)
    for perm in itertools.permutations(range(n)):
        val = C[rows, list(perm)].sum() / n
        if val < best:
            best = val
    return best


def w1_line_closed_form(f, g, h):
    """W1 between f and g on points 0, h, 2h, ...: h * sum_k |F_k - G_k|."""
    F = np.cumsum(f)
    G = np.cumsum(g)
    return h * float(np.abs(F[:-1] - G[:-1]).sum())


def monotone_coupling(x, f, y, g, cost):
    """North-west-corner coupling of sorted 1-D supports; optimal for convex cost(x-y)."""
    ix = np.argsort(x, kind="stable")
    iy = np.argsort(y, kind="stable")
    a = np.array(f, dtype=np.float64)[ix]
    b = np.array(g, dtype=np.float64)[iy]
    i = j = 0
    total = 0.0
    while i < len(a) and j < len(b):
        t = min(a[i], b[j])
        total += t * cost(x[ix[i]] - y[iy[j]])
        a[i] -= t
        b[j] -= t
        if a[i] <= b[j]:
            i += 1
        else:
            j += 1
    return total
