"""Pins for the CPU oracle: checks against what the paper and mathematics fix, not against itself.

* the paper's worked example (Section 3.1) and Equation 2 by hand  -> golden/paper_triangle.json
* a literal brute force of the pairing rules on the Kuhn triangulation (oracle/brute.py)
* the Euler characteristic of a box (chi = 1), closed-form cell counts
* exact rational arithmetic for the floors and the quantized edit
* the problem statement's postconditions: |g - f| <= xi, decrease-only edits, MSC equality
* the paper's per-case choice of which vertex to lower (Sections 4.3-4.4)
"""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2409_17346_amd import synth

from floorcheck import collision_field, explained

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _pairs_from_oracle(cx, up):
    out = set()
    for d in range(cx.top):
        for i, u in enumerate(up[d]):
            if u >= 0:
                out.add((frozenset(cx.vertices(d, i)), frozenset(cx.vertices(d + 1, int(u)))))
    return out


def _crit_from_oracle(cx, up, dn):
    crit = []
    for d in range(cx.top + 1):
        ex = cx.exists(d)
        s = set()
        for i in range(cx.ncell[d]):
            if ex[i] and up[d][i] < 0 and dn[d][i] < 0:
                s.add(frozenset(cx.vertices(d, i)))
        crit.append(s)
    return crit


# ------------------------------------------------------------------------------------------
# Worked example of Section 3.1 (+ Equation 2 by hand)

def test_paper_triangle_example():
    g = json.load(open(os.path.join(GOLD, "paper_triangle.json")))
    cx = oracle.Complex.explicit(2, 3, edges=sum(g["edges"], []), tris=sum(g["triangles"], []))
    f = np.array(g["f"], np.float32)
    fh = np.array(g["f_hat"], np.float32)
    for field, pk, ck in ((f, "f_pairs", "f_critical"), (fh, "f_hat_pairs", "f_hat_critical")):
        up, dn = oracle.gradient(cx, field)
        assert _pairs_from_oracle(cx, up) == {(frozenset(a), frozenset(b)) for a, b in g[pk]}
        crit = set().union(*_crit_from_oracle(cx, up, dn))
        assert crit == {frozenset(c) for c in g[ck]}
    # first iteration: FPmin at j and FNmin at k, both fixed by lowering k
    r1 = oracle.correct(cx, f, fh, g["xi"], 4, g["q_max"], max_iters=1)
    assert r1["log"][0][1] == g["first_iteration"]["FP0"] and r1["log"][0][2] == g["first_iteration"]["FN0"]
    assert sorted(np.nonzero(r1["q"])[0].tolist()) == g["first_iteration"]["requested"]
    # trajectory of g_k, one iteration at a time
    traj = [float(oracle.correct(cx, f, fh, g["xi"], 4, g["q_max"], max_iters=k)["g"][2]) for k in range(1, 8)]
    assert traj == g["g_trajectory_k"]
    r = oracle.correct(cx, f, fh, g["xi"], 4, g["q_max"])
    assert r["status"] == "ok"
    assert r["g"].tolist() == g["final_g"]
    assert r["q"].tolist() == g["final_q"]
    assert [[int(i), float(v)] for i, v in zip(r["lossless_idx"], r["lossless_val"])] == g["lossless"]
    assert r["stats"]["c_iterations"] == g["c_iterations"] and r["stats"]["s_iterations"] == g["s_iterations"]


# ------------------------------------------------------------------------------------------
# Gradient and MSC vs the literal brute force

SHAPES = [(3, 3), (4, 3), (3, 5), (5, 4), (3, 3, 3), (4, 3, 3), (3, 4, 4)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", ["uniform", "plateau", "perm", "const"])
def test_gradient_matches_brute_force(shape, kind):
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) == 3 else 1
    cx = oracle.Complex.grid(nx, ny, nz)
    cells = brute.kuhn_complex(shape)
    assert [len(c) for c in cells] == [int(cx.exists(d).sum()) for d in range(cx.top + 1)]
    for seed in range(12 if kind != "const" else 1):
        h = synth.random_field((nz, ny, nx) if nz > 1 else (ny, nx), kind, seed).reshape(-1)
        up, dn = oracle.gradient(cx, h)
        pair, crit, _ = brute.gradient(cells, h)
        assert _pairs_from_oracle(cx, up) == {(a, b) for a, b in pair.items() if len(a) < len(b)}
        assert _crit_from_oracle(cx, up, dn) == crit


def test_gradient_all_orderings_3x3_sample():
    """A spread-out sample of all 9! vertex orderings of the 3x3 grid."""
    cx = oracle.Complex.grid(3, 3, 1)
    cells = brute.kuhn_complex((3, 3))
    perms = list(itertools.permutations(range(9)))
    for p in perms[:: len(perms) // 1500]:
        h = np.array(p, np.float32)
        up, dn = oracle.gradient(cx, h)
        pair, crit, _ = brute.gradient(cells, h)
        assert _pairs_from_oracle(cx, up) == {(a, b) for a, b in pair.items() if len(a) < len(b)}


def _oracle_msc_as_sets(cx, h):
    m = oracle.msc(cx, h)
    top = cx.top
    crit = [set(frozenset(cx.vertices(d, int(i))) for i in m.crit[d]) for d in range(top + 1)]
    desc = set()
    for b in range(len(m.desc_saddle)):
        seq = tuple(int(v) for v in m.desc_cells[m.desc_offsets[b]:m.desc_offsets[b + 1]])
        desc.add((frozenset(cx.vertices(1, int(m.desc_saddle[b]))), seq))
        assert seq[-1] == m.desc_terminal[b]
    asc = set()
    for b in range(len(m.asc_saddle)):
        seq = tuple(frozenset(cx.vertices(top, int(t))) for t in m.asc_cells[m.asc_offsets[b]:m.asc_offsets[b + 1]])
        term = None if m.asc_terminal[b] < 0 else frozenset(cx.vertices(top, int(m.asc_terminal[b])))
        asc.add((frozenset(cx.vertices(top - 1, int(m.asc_saddle[b]))), seq, term))
    return crit, desc, asc, m


@pytest.mark.parametrize("shape", [(4, 4), (6, 5), (3, 3, 3), (4, 4, 3)])
@pytest.mark.parametrize("kind", ["uniform", "plateau", "smooth"])
def test_msc_matches_brute_force(shape, kind):
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) == 3 else 1
    cx = oracle.Complex.grid(nx, ny, nz)
    cells = brute.kuhn_complex(shape)
    for seed in range(6):
        h = synth.random_field((nz, ny, nx) if nz > 1 else (ny, nx), kind, seed).reshape(-1)
        crit, desc, asc, m = _oracle_msc_as_sets(cx, h)
        b = brute.msc(cells, h)
        assert crit == b["crit"]
        assert desc == b["desc"]
        assert asc == b["asc"]
        # labels: terminal of every cell's own V-path
        for v in range(cx.nv):
            path = [v]
            cur = frozenset([v])
            while cur in b["pair"]:
                (w,) = tuple(b["pair"][cur] - cur)
                cur = frozenset([w])
            assert m.min_label[v] == min(cur)
        # max labels: terminal of every top cell's own ascending V-path (BOUNDARY = -1); ids of
        # top cells that leave the grid read -2
        top = cx.top
        ids = {frozenset(cx.vertices(top, t)): t for t in range(cx.ncell[top]) if cx.vertices(top, t)}
        _, _, cof = brute.gradient(cells, h)
        assert len(m.max_label) == cx.ncell[top]
        for t in range(cx.ncell[top]):
            vs = cx.vertices(top, t)
            if vs is None:
                assert m.max_label[t] == -2
                continue
            T = frozenset(vs)
            term = T
            while term is not None and term in b["pair"]:
                others = [c for c in cof[b["pair"][term]] if c != term]
                term = others[0] if others else None
            assert m.max_label[t] == (-1 if term is None else ids[term]), (t, vs)


# ------------------------------------------------------------------------------------------
# Euler characteristic and cell counts

def _euler(cx, h):
    m = oracle.msc(cx, h)
    return sum((-1) ** d * len(m.crit[d]) for d in range(cx.top + 1))


@pytest.mark.parametrize("dims", [(17, 13, 1), (2, 2, 1), (32, 2, 1), (7, 6, 5), (2, 2, 2), (9, 3, 4)])
def test_euler_characteristic_is_one(dims):
    nx, ny, nz = dims
    cx = oracle.Complex.grid(nx, ny, nz)
    shape = (nz, ny, nx) if nz > 1 else (ny, nx)
    for kind in ("uniform", "plateau", "smooth", "const", "perm"):
        for seed in range(3):
            assert _euler(cx, synth.random_field(shape, kind, seed).reshape(-1)) == 1


def test_cell_counts_closed_form():
    # 2D n x m: V = nm, E = 3nm - 2n - 2m + 1, T = 2(n-1)(m-1); 3D (n^3): Kuhn counts
    for n, m in [(2, 2), (5, 3), (17, 9)]:
        cx = oracle.Complex.grid(n, m, 1)
        e = [int(cx.exists(d).sum()) for d in range(3)]
        assert e == [n * m, 3 * n * m - 2 * n - 2 * m + 1, 2 * (n - 1) * (m - 1)]
    for n in (2, 3, 5):
        cx = oracle.Complex.grid(n, n, n)
        e = [int(cx.exists(d).sum()) for d in range(4)]
        c = (n - 1) ** 3
        sq = 3 * n * (n - 1) ** 2
        ln = 3 * n * n * (n - 1)
        # edges: axis + face diagonals (one per square) + body diagonals (one per cube)
        assert e[1] == ln + sq + c
        # triangles: 2 per square + 6 interior per cube; tets: 6 per cube
        assert e[2] == 2 * sq + 6 * c
        assert e[3] == 6 * c
        assert e[0] - e[1] + e[2] - e[3] == 1


def test_constant_field_single_critical_cell():
    for dims in [(6, 5, 1), (4, 3, 3)]:
        cx = oracle.Complex.grid(*dims)
        m = oracle.msc(cx, np.zeros(cx.nv, np.float32))
        assert [len(c) for c in m.crit] == [1] + [0] * cx.top
        assert m.crit[0][0] == 0


# ------------------------------------------------------------------------------------------
# Exact arithmetic: floors, ceilings and the quantized edit

def _f32_neighbours(x):
    x = np.float32(x)
    return [np.nextafter(x, np.float32(-np.inf)), x, np.nextafter(x, np.float32(np.inf))]


def test_bounds_exact_rational():
    rng = np.random.default_rng(5)
    vals = np.concatenate([rng.uniform(-2, 2, 300), rng.uniform(-1e-6, 1e-6, 50), [0.0, -0.0, 1e-4, 1.0, 3.0],
                           np.float32(1e-38) * rng.uniform(0, 1, 20)]).astype(np.float32)
    for xi in (np.float32(1e-4), np.float32(0.37), np.float32(1.0), np.float32(3e-39)):
        lo, hi = oracle.bounds(vals, float(xi))
        for f, l, h in zip(vals, lo, hi):
            ex_lo = Fraction(float(f)) - Fraction(float(xi))
            ex_hi = Fraction(float(f)) + Fraction(float(xi))
            assert Fraction(float(l)) >= ex_lo
            assert Fraction(float(np.nextafter(l, np.float32(-np.inf)))) < ex_lo
            assert Fraction(float(h)) <= ex_hi
            assert Fraction(float(np.nextafter(h, np.float32(np.inf)))) > ex_hi


def _round_nearest_even_f32(fr: Fraction) -> np.float32:
    best = None
    for c in _f32_neighbours(float(fr)):
        d = abs(Fraction(float(c)) - fr)
        if best is None or d < best[0] or (d == best[0] and (int(c.view(np.uint32)) & 1) == 0):
            best = (d, c)
    return best[1]


def test_quantized_edit_is_one_rounding():
    """g = g_hat - q * xi / 2^q_max rounded once to nearest-even (decoder path)."""
    rng = np.random.default_rng(9)
    gh = np.concatenate([rng.uniform(-1, 1, 200), rng.uniform(0, 1e-3, 50)]).astype(np.float32)
    for xi, qmax in ((np.float32(1e-4), 6), (np.float32(0.3), 2), (np.float32(1.0), 7)):
        for q in range(0, qmax + 1):
            qa = np.full(gh.size, q, np.uint8)
            out = oracle.decode(gh, qa, np.zeros(0, np.int64), np.zeros(0, np.float32), float(xi), qmax)
            delta = Fraction(float(xi)) / (2 ** qmax)
            for a, o in zip(gh, out):
                exp = _round_nearest_even_f32(Fraction(float(a)) - q * delta)
                assert o.view(np.uint32) == exp.view(np.uint32) or (o == 0 and exp == 0)


# ------------------------------------------------------------------------------------------
# Postconditions of the problem statement and the convergence argument

def _exact_within(f, g, xi):
    for a, b in zip(f.reshape(-1), g.reshape(-1)):
        assert abs(Fraction(float(a)) - Fraction(float(b))) <= Fraction(float(xi))


def _assert_floor_collision_stall(cx, dims, f, g, xi, tier, n_residual):
    """Every violation left at a stall has an equal-floor inverted pair of floored vertices in the
    closed 1-ring of its highest vertex (the only way decrease-only edits can get stuck)."""
    res = oracle.residual(cx, f, g, tier)
    assert len(res) == n_residual
    lo, _ = oracle.bounds(f, xi)
    ok = explained(dims, f, g, lo, res)
    assert ok.all(), res[~ok][:8]


def _cases():
    out = []
    for shape in [(8, 8), (12, 9), (5, 5, 4)]:
        for kind in ["uniform", "plateau", "smooth"]:
            for ghat in ["noise", "bin"]:
                for seed in range(2):
                    out.append((shape, kind, ghat, seed))
    return out


@pytest.mark.parametrize("shape,kind,ghat,seed", _cases())
def test_correction_postconditions(shape, kind, ghat, seed):
    w = synth.tiny_cases(seed, shape, rel=0.2, kind=kind, ghat=ghat)
    nx, ny, nz = w.dims
    cx = oracle.Complex.grid(nx, ny, nz)
    f = w.f.reshape(-1)
    gh = w.g_hat.reshape(-1)
    cells = brute.kuhn_complex((nx, ny) if nz == 1 else (nx, ny, nz))
    bf = brute.msc(cells, f)
    for tier in (1, 2, 3, 4):
        r = oracle.correct(cx, f, gh, w.xi, tier, 6)
        st = r["stats"]
        assert r["status"] in ("ok", "not_converged")
        g = r["g"]
        _exact_within(f, g, w.xi)
        assert np.all(g <= gh)
        # decoder round trip
        dec = oracle.decode(gh, r["q"], r["lossless_idx"], r["lossless_val"], w.xi, 6)
        assert np.array_equal(dec.view(np.uint32), g.view(np.uint32))
        # termination bound of the convergence argument: each vertex moves at most q_max+1 times
        assert st["iterations"] <= cx.nv * 7
        assert st["n_edited"] == st["n_quantized"] + st["n_lossless"]
        if r["status"] != "ok":
            assert st["stalled"] == 1 and st["residual_violations"] > 0
            _assert_floor_collision_stall(cx, w.dims, f, g, w.xi, tier, st["residual_violations"])
            continue
        bg = brute.msc(cells, g)
        n = cx.top
        if tier == 1:
            assert bg["crit"][0] == bf["crit"][0] and bg["crit"][n] == bf["crit"][n]
        else:
            assert bg["crit"] == bf["crit"]
        if tier == 3:
            assert {(s, p[0], p[-1]) for s, p in bg["desc"]} == {(s, p[0], p[-1]) for s, p in bf["desc"]}
            assert {(s, p[0], t) for s, p, t in bg["asc"]} == {(s, p[0], t) for s, p, t in bf["asc"]}
        if tier == 4:
            assert bg["desc"] == bf["desc"] and bg["asc"] == bf["asc"]


def test_trajectory_is_monotone_and_bounded():
    w = synth.tiny_cases(3, (10, 10), rel=0.3, kind="uniform", ghat="noise")
    cx = oracle.Complex.grid(10, 10, 1)
    f, gh = w.f.reshape(-1), w.g_hat.reshape(-1)
    full = oracle.correct(cx, f, gh, w.xi, 4, 6)
    lo, hi = oracle.bounds(f, w.xi)
    prev = gh.copy()
    for k in range(1, full["stats"]["iterations"] + 1):
        g = oracle.correct(cx, f, gh, w.xi, 4, 6, max_iters=k)["g"]
        assert np.all(g <= prev) and np.all(g >= lo)
        prev = g
    assert np.array_equal(prev, full["g"])


def test_identity_and_floor_inputs():
    w = synth.tiny_cases(1, (9, 7), rel=0.1, kind="uniform")
    cx = oracle.Complex.grid(9, 7, 1)
    f = w.f.reshape(-1)
    r = oracle.correct(cx, f, f, w.xi, 4, 6)
    assert r["status"] == "ok" and r["stats"]["iterations"] == 0 and r["stats"]["n_edited"] == 0
    assert np.array_equal(r["g"].view(np.uint32), f.view(np.uint32))
    lo, _ = oracle.bounds(f, w.xi)
    r = oracle.correct(cx, f, lo, w.xi, 4, 6)
    # every vertex at its floor: the order of the floors is f's order unless two floors collide
    if len(np.unique(lo)) == lo.size and np.array_equal(np.argsort(lo, kind="stable"), np.argsort(f, kind="stable")):
        assert r["stats"]["n_edited"] == 0


def test_error_statuses():
    cx = oracle.Complex.grid(4, 4, 1)
    f = np.linspace(0, 1, 16, dtype=np.float32)
    assert oracle.correct(cx, f, f + np.float32(0.5), 0.1)["status"] == "bound"
    bad = f.copy()
    bad[3] = np.nan
    assert oracle.correct(cx, bad, f, 0.1)["status"] == "nonfinite"
    assert oracle.correct(cx, f, f, 0.0)["status"] == "invalid"
    assert oracle.correct(cx, f, f, 0.1, tier=5)["status"] == "invalid"
    assert oracle.correct(cx, f, f, 1e-37, q_max=7)["status"] == "invalid"   # Delta subnormal


# ------------------------------------------------------------------------------------------
# Which vertex gets lowered: the paper's case analysis (Sections 4.3, 4.4)

def _allowed_targets(cells, pf, pg, f, key):
    """Per violating cell, the set of vertices the paper allows lowering, from its text:
    FPmin -> j (the f-partner's other vertex); FPmax -> the vertex the f-pair adds; FP saddles ->
    a vertex of the cell paired with it in f; FN (paired in g as (sigma, tau)) -> a vertex of
    sigma ("decrease i", "i or j", "i, j or k")."""
    def lt(a, b):
        return (f[a], key[a]) < (f[b], key[b])
    n = len(cells) - 1
    out = []
    for d in range(n + 1):
        for c in cells[d]:
            fc, gc = c not in pf, c not in pg
            if fc == gc:
                continue
            if not fc:
                p = pf[c]
                hi_, lo_ = (p, c) if len(p) > len(c) else (c, p)
                apex = next(iter(hi_ - lo_))
                out.append({apex} if d in (0, n) else set(hi_))
            else:
                p = pg[c]
                hi_, lo_ = (p, c) if len(p) > len(c) else (c, p)
                x = next(iter(hi_ - lo_))
                if any(lt(w, x) for w in lo_):
                    out.append(set(lo_))
                else:
                    out.append(None)   # orientation the paper does not depict
    return out


@pytest.mark.parametrize("top", [2, 3])
def test_first_step_targets_follow_paper_cases(top):
    cells = brute.explicit_complex([[0, 1, 2]] if top == 2 else [[0, 1, 2, 3]])
    nv = top + 1
    edges = [sorted(c) for c in cells[1]]
    tris = [sorted(c) for c in cells[2]]
    tets = [sorted(c) for c in cells[3]] if top == 3 else []
    cx = oracle.Complex.explicit(top, nv, edges=sum(edges, []), tris=sum(tris, []), tets=sum(tets, []))
    key = np.arange(nv)
    checked = 0
    for pf_ in itertools.permutations(range(nv)):
        for pg_ in itertools.permutations(range(nv)):
            f = np.array(pf_, np.float32)
            gh = np.array(pg_, np.float32)
            allowed = _allowed_targets(cells, brute.gradient(cells, f)[0], brute.gradient(cells, gh)[0], f, key)
            r = oracle.correct(cx, f, gh, float(nv), 2, 6, max_iters=1)
            R = set(np.nonzero(r["q"] != 0)[0].tolist())
            if not allowed:
                assert not R
                continue
            if any(a is None for a in allowed):
                continue
            union = set().union(*allowed)
            assert R <= union, (pf_, pg_, R, allowed)
            for a in allowed:
                assert R & a, (pf_, pg_, R, allowed)
            checked += 1
    assert checked > 10


@pytest.mark.parametrize("dims", [(7, 6, 1), (5, 5, 4)])
def test_troublemaker_targets_follow_paper(dims):
    """S-loop targets (Section 4.4): a vertex i paired with ik in g but ij in f -> lower j (0-dim
    troublemaker); a top cell paired with a different facet in g than in f -> lower the vertex its
    f-facet lacks (2D: triangle ijk paired with edge ij in f; 3D, TM2: triangle ijk paired with
    ijkl in f but ijkq in g -> lower l)."""
    rng = np.random.default_rng(11)
    nx, ny, nz = dims
    shape = (ny, nx) if nz == 1 else (nz, ny, nx)
    cx = oracle.Complex.grid(nx, ny, nz)
    cells = brute.kuhn_complex((nx, ny) if nz == 1 else (nx, ny, nz))
    found = 0
    for trial in range(60):
        f = synth.random_field(shape, "smooth", trial).reshape(-1)
        xi = float(np.float32(0.15 * (f.max() - f.min())))
        gh = synth.uniform_noise(f, xi, rng)
        r0 = oracle.correct(cx, f, gh, xi, 4, 6)
        if r0["status"] != "ok":
            continue
        log = r0["log"]
        s_rows = [k for k in range(len(log)) if log[k][0] == 2]
        if not s_rows:
            continue
        k = s_rows[0]
        g_before = oracle.correct(cx, f, gh, xi, 4, 6, max_iters=k)["g"]
        g_after = oracle.correct(cx, f, gh, xi, 4, 6, max_iters=k + 1)["g"]
        R = set(np.nonzero(g_after != g_before)[0].tolist())
        bf = brute.msc(cells, f)
        pf = bf["pair"]
        pg = brute.gradient(cells, g_before)[0]
        allowed = set()
        for _, seq in bf["desc"]:
            for v in seq:
                c = frozenset([v])
                if pf.get(c) != pg.get(c):
                    allowed |= set(pf[c] - c)
                    break
        for _, seq, _t in bf["asc"]:
            for T in seq:
                if pf.get(T) != pg.get(T):
                    allowed |= set(T - pf[T])
                    break
        assert R and R <= allowed
        found += 1
    assert found >= 3


def _brute_residual(cells, f, g, tier):
    """Violating cells from the brute force: criticality differences (tier filter), else the first
    differing cell of each separatrix branch (tier 3: only branches whose g-path ends elsewhere)."""
    n = len(cells) - 1
    pf, critf, cof = brute.gradient(cells, f)
    pg, critg, _ = brute.gradient(cells, g)
    out = [c for d in range(n + 1) if not (tier == 1 and d not in (0, n))
           for c in cells[d] if (c in critf[d]) != (c in critg[d])]
    if out or tier < 3:
        return out

    def end_desc(v):
        cur = frozenset([v])
        while cur in pg:
            (w,) = tuple(pg[cur] - cur)
            cur = frozenset([w])
        return min(cur)

    def end_asc(T):
        while T in pg:
            others = [x for x in cof[pg[T]] if x != T]
            if not others:
                return None
            T = others[0]
        return T

    bf = brute.msc(cells, f)
    for _, seq in sorted(bf["desc"], key=lambda x: (sorted(x[0]), x[1])):
        for v in seq:
            c = frozenset([v])
            if pf.get(c) != pg.get(c):
                if tier == 4 or end_desc(seq[0]) != seq[-1]:
                    out.append(c)
                break
    for _, seq, t in bf["asc"]:
        for T in seq:
            if pf.get(T) != pg.get(T):
                if tier == 4 or end_asc(seq[0]) != t:
                    out.append(T)
                break
    return out


@pytest.mark.parametrize("dims", [(6, 5, 1), (4, 4, 3)])
def test_residual_list_matches_brute_force(dims):
    """oracle.residual lists the violations the loop would fix: checked as a multiset of cells
    against the brute force on g_hat and on partly corrected fields, at every tier."""
    nx, ny, nz = dims
    shape = (ny, nx) if nz == 1 else (nz, ny, nx)
    cx = oracle.Complex.grid(nx, ny, nz)
    cells = brute.kuhn_complex((nx, ny) if nz == 1 else (nx, ny, nz))
    checked = 0
    for seed in range(8):
        w = synth.tiny_cases(seed, shape, rel=0.2, kind="smooth", ghat="noise")
        f, gh = w.f.reshape(-1), w.g_hat.reshape(-1)
        for tier in (1, 2, 3, 4):
            for k in (0, 2, 5):
                g = oracle.correct(cx, f, gh, w.xi, tier, 6, max_iters=k)["g"]
                res = oracle.residual(cx, f, g, tier)
                mine = sorted(tuple(sorted(cx.vertices(int(d), int(i)))) for d, i in res)
                ref = sorted(tuple(sorted(c)) for c in _brute_residual(cells, f, g, tier))
                assert mine == ref
                checked += len(ref) > 0
    assert checked > 20


@pytest.mark.parametrize("dims", [(6, 6, 1), (8, 7, 1), (4, 4, 4), (5, 4, 3)])
def test_stalls_are_floor_collisions(dims):
    """Fields built so that many floors collide (xi = 1, most values below 2^-24) stall; every
    violation left behind is explained by an equal-floor inverted pair at the floors, and the
    violations reported match the oracle's residual count."""
    nx, ny, nz = dims
    shape = (ny, nx) if nz == 1 else (nz, ny, nx)
    cx = oracle.Complex.grid(nx, ny, nz)
    stalls = 0
    for seed in range(12):
        f, rng = collision_field(shape, seed)
        gh = synth.uniform_noise(f, 1.0, rng)
        f, gh = f.reshape(-1), gh.reshape(-1)
        for tier in (1, 2, 4):
            r = oracle.correct(cx, f, gh, 1.0, tier, 6)
            if r["status"] == "ok":
                continue
            assert r["stats"]["stalled"] == 1
            _assert_floor_collision_stall(cx, (nx, ny, nz), f, r["g"], 1.0, tier,
                                          r["stats"]["residual_violations"])
            stalls += 1
    assert stalls >= 6


def test_floor_collision_check_rejects_other_stalls():
    """The stall check is not vacuous: without floor collisions (distinct, well separated floors)
    an unexplained violation is reported as such."""
    nx, ny = 6, 5
    cx = oracle.Complex.grid(nx, ny, 1)
    f = synth.random_field((ny, nx), "perm", 3).reshape(-1)       # integers, floors never collide
    gh = f[::-1].copy()                                          # every order reversed
    res = oracle.residual(cx, f, gh, 2)
    assert len(res) > 0
    lo, _ = oracle.bounds(f, 100.0)
    assert not explained((nx, ny, 1), f, gh, lo, res).any()


# ------------------------------------------------------------------------------------------
# Verification metrics (Section 5.1): agreement of two complexes

def _brute_agreement(cells, f, g):
    """Agreement counts from two brute-force complexes (cells as vertex sets, separatrices keyed
    by their saddle and first cell)."""
    bf, bg = brute.msc(cells, f), brute.msc(cells, g)
    n = len(cells) - 1
    out = {"crit_f": [0] * 4, "crit_g": [0] * 4, "crit_common": [0] * 4}
    for d in range(n + 1):
        a, b = set(bf["crit"][d]), set(bg["crit"][d])
        out["crit_f"][d], out["crit_g"][d], out["crit_common"][d] = len(a), len(b), len(a & b)

    def desc(m):
        return {(e, p[0]): (p[-1], p) for e, p in m["desc"]}

    def asc(m):
        return {(s, p[0]): (t, p) for s, p, t in m["asc"]}

    out.update(sep_f=[0, 0], sep_g=[0, 0], sep_same_ends=[0, 0], sep_same_cells=[0, 0])
    for k, fam in enumerate((desc, asc)):
        sf, sg = fam(bf), fam(bg)
        out["sep_f"][k], out["sep_g"][k] = len(sf), len(sg)
        for key, (t, p) in sf.items():
            if key in sg:
                out["sep_same_ends"][k] += sg[key][0] == t
                out["sep_same_cells"][k] += sg[key] == (t, p)
    return out


@pytest.mark.parametrize("shape", [(5, 4), (7, 6), (3, 3, 3), (4, 3, 3)])
def test_agreement_matches_brute_force(shape):
    """The oracle's agreement counts equal those of two brute-force complexes, for g_hat (which
    changes the complex) and for corrections at tiers 1-3 (which restore parts of it)."""
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) == 3 else 1
    cx = oracle.Complex.grid(nx, ny, nz)
    cells = brute.kuhn_complex(shape)
    seen_partial = False
    for seed in range(5):
        w = synth.tiny_cases(seed, (nz, ny, nx) if nz > 1 else (ny, nx), rel=0.2, kind="uniform", ghat="noise")
        f, gh = w.f.reshape(-1), w.g_hat.reshape(-1)
        gs = [gh] + [oracle.correct(cx, f, gh, w.xi, t, 6)["g"] for t in (1, 2, 3)]
        for g in gs:
            a = oracle.msc_agreement(cx, f, g)
            assert a == _brute_agreement(cells, f, g)
            seen_partial |= sum(a["crit_common"]) < sum(a["crit_f"])
    assert seen_partial


@pytest.mark.parametrize("dims", [(12, 9, 1), (6, 5, 4)])
def test_agreement_invariants(dims):
    """The complex depends only on the order of the values: any increasing transform of f agrees
    with f in full; the counts are symmetric in f and g; a field corrected at tier t agrees with f
    in critical cells (t >= 2), separatrix ends (t >= 3) and separatrix cells (t = 4)."""
    nx, ny, nz = dims
    cx = oracle.Complex.grid(nx, ny, nz)
    shape = (nz, ny, nx) if nz > 1 else (ny, nx)
    for seed in range(4):
        w = synth.tiny_cases(seed, shape, rel=0.05, kind="smooth", ghat="noise")
        f, gh = w.f.reshape(-1).astype(np.float64), w.g_hat.reshape(-1)
        for g in (f + 3.0, 2.0 * f - 1.0, np.cbrt(f + 0.25)):
            a = oracle.msc_agreement(cx, f, g.astype(np.float32))
            assert a["crit_common"] == a["crit_f"] == a["crit_g"]
            assert a["sep_same_cells"] == a["sep_same_ends"] == a["sep_f"] == a["sep_g"]
        a, b = oracle.msc_agreement(cx, f, gh), oracle.msc_agreement(cx, gh, f)
        assert a["crit_common"] == b["crit_common"] and a["crit_f"] == b["crit_g"]
        assert a["sep_same_cells"] == b["sep_same_cells"] and a["sep_same_ends"] == b["sep_same_ends"]
        for tier in (2, 3, 4):
            o = oracle.correct(cx, f, gh, w.xi, tier, 6)
            if o["status"] != "ok":
                continue
            a = oracle.msc_agreement(cx, f, o["g"])
            assert a["crit_common"] == a["crit_f"] == a["crit_g"]
            if tier >= 3:
                assert a["sep_same_ends"] == a["sep_f"] == a["sep_g"]
            if tier == 4:
                assert a["sep_same_cells"] == a["sep_f"]


# ------------------------------------------------------------------------------------------
# Edit stream (Section 4.7): fixed-bit codes, lossless values in vertex order

def test_edit_stream_hand_examples():
    assert [oracle.edit_bits(q) for q in range(8)] == [1, 2, 2, 3, 3, 3, 3, 4]
    # q_max 6: 3-bit codes, the 11th code (lossless = 7) straddles the first word boundary:
    # 1 + 2*8 + 7*64 + 5*4096 + 6*32768 + 3*262144 + (7 << 30 mod 2^32) = 3222229457, then bit 32 = 1
    assert oracle.pack_edits([1, 2, 0xFF, 0, 5, 6, 3, 0, 0, 0, 0xFF], 6).tolist() == [3222229457, 1]
    # q_max 0: 1-bit codes, alternating 0 / lossless
    assert oracle.pack_edits([0, 0xFF] * 18, 0).tolist() == [0xAAAAAAAA, 0b1010]
    # q_max 7: 4-bit codes, lossless = 8
    assert oracle.pack_edits([7, 0xFF, 1], 7).tolist() == [7 | 8 << 4 | 1 << 8]


@pytest.mark.parametrize("q_max", range(8))
def test_edit_stream_round_trip(q_max):
    rng = np.random.default_rng(q_max)
    for n in (1, 31, 32, 33, 1000, 4099):
        q = rng.integers(0, q_max + 2, size=n).astype(np.uint8)
        q[q == q_max + 1] = 0xFF
        words = oracle.pack_edits(q, q_max)
        assert len(words) == (n * oracle.edit_bits(q_max) + 31) // 32
        assert np.array_equal(oracle.unpack_edits(words, n, q_max), q)


def test_edit_stream_decodes_a_correction():
    """Stream + lossless values in vertex order reproduce the corrected field bit for bit."""
    w = synth.config_small2d()
    cx = oracle.Complex.grid(*w.dims)
    o = oracle.correct(cx, w.f.reshape(-1), w.g_hat.reshape(-1), w.xi, 4, 6)
    q = oracle.unpack_edits(oracle.pack_edits(o["q"], 6), len(o["q"]), 6)
    idx = np.nonzero(q == 0xFF)[0]
    g = oracle.decode(w.g_hat.reshape(-1), q, idx, o["g"][idx], w.xi, 6)
    assert np.array_equal(g.view(np.uint32), o["g"].view(np.uint32))


# ------------------------------------------------------------------------------------------
# Saddle-saddle connectors (3D, Section 3.1 / Section 4.4 1-dimensional troublemakers)

SS_CASES = [((5, 4, 4), "smooth", 0), ((5, 4, 4), "smooth", 8), ((5, 5, 4), "smooth", 4),
            ((5, 5, 4), "smooth", 10), ((6, 5, 4), "uniform", 6), ((6, 5, 4), "smooth", 10),
            ((4, 4, 4), "uniform", 3), ((5, 5, 5), "uniform", 1)]


@pytest.mark.parametrize("shape,kind,seed", SS_CASES)
def test_saddle_saddle_troublemakers_match_brute_force(shape, kind, seed):
    """On a field whose critical cells already agree with f (a tier-2 correction), the oracle's
    saddle-saddle troublemakers are the edges a literal walk of the brute-force 1-2 V-paths finds."""
    nx, ny, nz = shape
    cx = oracle.Complex.grid(nx, ny, nz)
    cells = brute.kuhn_complex(shape)
    w = synth.tiny_cases(seed, (nz, ny, nx), rel=0.2, kind=kind, ghat="noise")
    f = w.f.reshape(-1)
    g2 = oracle.correct(cx, f, w.g_hat.reshape(-1), w.xi, 2, 6)["g"]
    res = oracle.residual(cx, f, g2, 4, saddle_saddle=True)
    ids = {frozenset(cx.vertices(1, e)): e for e in range(cx.ncell[1]) if cx.vertices(1, e)}
    assert set(int(i) for d, i in res if d == 1) == {ids[e] for e in brute.ss_troublemakers(cells, f, g2)}


@pytest.mark.parametrize("shape,kind,seed", SS_CASES[:6])
def test_saddle_saddle_connectors_preserved(shape, kind, seed):
    """With the saddle-saddle option a converged tier-4 correction has exactly f's connectors
    (every V-path from a 2-saddle to a 1-saddle, enumerated by brute force); the listed cases are
    ones where tier 4 without the option leaves some connector different."""
    nx, ny, nz = shape
    cx = oracle.Complex.grid(nx, ny, nz)
    cells = brute.kuhn_complex(shape)
    w = synth.tiny_cases(seed, (nz, ny, nx), rel=0.2, kind=kind, ghat="noise")
    f, gh = w.f.reshape(-1), w.g_hat.reshape(-1)
    cf = brute.connectors(cells, f)
    o = oracle.correct(cx, f, gh, w.xi, 4, 6, saddle_saddle=True)
    assert o["status"] == "ok"
    assert brute.connectors(cells, o["g"]) == cf
    assert brute.msc(cells, o["g"])["desc"] == brute.msc(cells, f)["desc"]
    assert o["log"][:, 13].sum() > 0 or len(cf) == 0
    plain = oracle.correct(cx, f, gh, w.xi, 4, 6)
    assert plain["status"] == "ok" and brute.connectors(cells, plain["g"]) != cf
    # the option changes nothing in 2D or below tier 4
    if seed == 0:
        w2 = synth.tiny_cases(seed, (9, 8), rel=0.2, kind=kind, ghat="noise")
        cx2 = oracle.Complex.grid(8, 9, 1)
        a = oracle.correct(cx2, w2.f, w2.g_hat, w2.xi, 4, 6, saddle_saddle=True)
        b = oracle.correct(cx2, w2.f, w2.g_hat, w2.xi, 4, 6)
        assert np.array_equal(a["g"].view(np.uint32), b["g"].view(np.uint32))
        a = oracle.correct(cx, f, gh, w.xi, 3, 6, saddle_saddle=True)
        b = oracle.correct(cx, f, gh, w.xi, 3, 6)
        assert np.array_equal(a["g"].view(np.uint32), b["g"].view(np.uint32))
