"""Generator of the per-class ERI device code (run at build time).

For a class (la lb | lc ld), la >= lb, lc >= ld, it emits straight-line HIP
device functions templated on the arithmetic type T (double, float):

  vrr_<cls>(F, geometry scalars, acc)  accumulate the primitive integrals
      [e0|f0]^(0), |e| in [la, la+lb], |f| in [lc, lc+ld], into acc[]
      (vertical recurrence of Obara and Saika; [00|00]^(m) = F[m], which the
      caller has already multiplied by the quartet prefactor);
  hrr_<cls>(acc, AB, CD, out)          horizontal recurrence of Head-Gordon
      and Pople on the contracted values: (a,b+1_i| = (a+1_i,b| + AB_i (a,b|
      on the bra and the same with CD on the ket; out[] is (ab|cd) row-major
      over lexicographic Cartesian components.

The split follows the paper's description of the recurrences (Section 2.2):
HRR moves angular momentum from b to a (and d to c), VRR lowers it at a or c
down to [00|00], which is evaluated analytically.  The contraction of Eq. 2
happens between the two: the HRR coefficients AB, CD do not depend on the
primitives.

The order in which the recurrence lowers angular momentum is chosen by the
greedy search of Section 6 (Algorithm 1): at each node, every candidate
position (bra or ket centre, Cartesian direction) is scored by
(new intermediates - reused intermediates) + lambda * (angular momentum left
at that position), and the cheapest is taken.  The generator tries a few
lambda values and keeps the path with the fewest floating-point operations.

Recurrence used, with p, q the bra and ket exponent sums, rho = pq/(p+q),
W = (pP + qQ)/(p+q):
  [e+1_i|f]^(m) = PA_i [e|f]^(m) + WP_i [e|f]^(m+1)
                  + e_i/(2p) ([e-1_i|f]^(m) - rho/p [e-1_i|f]^(m+1))
                  + f_i/(2(p+q)) [e|f-1_i]^(m+1)
  [e|f+1_i]^(m) = QC_i [e|f]^(m) + WQ_i [e|f]^(m+1)
                  + f_i/(2q) ([e|f-1_i]^(m) - rho/q [e|f-1_i]^(m+1))
                  + e_i/(2(p+q)) [e-1_i|f]^(m+1)
"""
from __future__ import annotations

import json
import os
import random
import sys
from dataclasses import dataclass, field

AX = "xyz"


def cart(l):
    out = []
    for i in range(l, -1, -1):
        for j in range(l - i, -1, -1):
            out.append((i, j, l - i - j))
    return out


def ncart(l):
    return (l + 1) * (l + 2) // 2


def cidx(t):
    """Index of a Cartesian triple inside its shell (lexicographic)."""
    return cart(sum(t)).index(tuple(t))


def sub(t, i, k=1):
    t = list(t)
    t[i] -= k
    return tuple(t)


def add(t, i, k=1):
    t = list(t)
    t[i] += k
    return tuple(t)


ZERO3 = (0, 0, 0)


# --------------------------------------------------------------------------
# VRR DAG with the greedy path choice
# --------------------------------------------------------------------------

@dataclass
class VNode:
    e: tuple
    f: tuple
    m: int
    side: str = ""        # 'b' (lower e) or 'k' (lower f) or '' for a base node
    axis: int = -1
    deps: dict = field(default_factory=dict)
    name: str = ""


class VRR:
    def __init__(self, la, lb, lc, ld, lam):
        self.la, self.lb, self.lc, self.ld = la, lb, lc, ld
        self.L = la + lb + lc + ld
        self.lam = lam
        self.nodes = {}
        self.order = []

    def _children(self, e, f, m, side, i):
        ch = {}
        if side == "b":
            e1 = sub(e, i)
            ch["x1"] = (e1, f, m)
            ch["x2"] = (e1, f, m + 1)
            if e1[i] > 0:
                e2 = sub(e1, i)
                ch["x3"] = (e2, f, m)
                ch["x4"] = (e2, f, m + 1)
            if f[i] > 0:
                ch["x5"] = (e1, sub(f, i), m + 1)
        else:
            f1 = sub(f, i)
            ch["x1"] = (e, f1, m)
            ch["x2"] = (e, f1, m + 1)
            if f1[i] > 0:
                f2 = sub(f1, i)
                ch["x3"] = (e, f2, m)
                ch["x4"] = (e, f2, m + 1)
            if e[i] > 0:
                ch["x5"] = (sub(e, i), f1, m + 1)
        return ch

    def need(self, e, f, m):
        key = (e, f, m)
        if key in self.nodes:
            return self.nodes[key]
        if e == ZERO3 and f == ZERO3:
            node = VNode(e, f, m, name=f"F[{m}]")
            self.nodes[key] = node
            return node
        if FIXED_PATH:
            # ablation: the textbook order, no search (ket first, then bra,
            # along the first axis with a non-zero exponent)
            side, t = ("k", f) if f != ZERO3 else ("b", e)
            i = next(j for j in range(3) if t[j] > 0)
            ch = self._children(e, f, m, side, i)
            deps = {k: self.need(*c) for k, c in ch.items()}
            node = VNode(e, f, m, side=side, axis=i, deps=deps)
            node.name = f"v{len(self.order)}"
            self.nodes[key] = node
            self.order.append(node)
            return node
        # Algorithm 1: score every position, keep the cheapest
        best = None
        for side, t in (("b", e), ("k", f)):
            for i in range(3):
                if t[i] == 0:
                    continue
                ch = self._children(e, f, m, side, i)
                r = sum(1 for c in ch.values() if c in self.nodes)
                n = len(ch) - r
                a = sum(t) - 1
                cost = (n - r) + self.lam * a
                # deterministic tie-break: prefer the bra, then x, y, z
                tb = (cost, 0 if side == "b" else 1, i)
                if best is None or tb < best[0]:
                    best = (tb, side, i, ch)
        _, side, i, ch = best
        deps = {}
        for k, c in ch.items():
            deps[k] = self.need(*c)
        node = VNode(e, f, m, side=side, axis=i, deps=deps)
        node.name = f"v{len(self.order)}"
        self.nodes[key] = node
        self.order.append(node)
        return node

    def targets(self):
        es = [t for l in range(self.la, self.la + self.lb + 1) for t in cart(l)]
        fs = [t for l in range(self.lc, self.lc + self.ld + 1) for t in cart(l)]
        return es, fs

    def build(self, targets=None):
        """Build the DAG for `targets` (default: every [e0|f0] of the class)."""
        es, fs = self.targets()
        pairs = [(e, f) for e in es for f in fs] if targets is None else list(targets)
        self.built_targets = list(pairs)
        # highest angular momentum first: large nodes pull in shared low nodes
        for e, f in sorted(pairs, key=lambda ef: -(sum(ef[0]) + sum(ef[1]))):
            self.need(e, f, 0)
        return es, fs

    def flops(self):
        """Floating-point operations per primitive quartet (FMA = 2):
        A*x1 (1) + W*x2 (2) [+ c*(x3 - r*x4) (4)] [+ c5*x5 (2)] per node,
        plus one add per accumulated target."""
        fl = 0
        for n in self.order:
            d = n.deps
            fl += 3
            if "x3" in d:
                fl += 4
            if "x5" in d:
                fl += 2
        return fl + len(self.built_targets)


LAMBDAS = (0.0, 0.5, 1.0, 2.0, 4.0)
# MJK_FIXED_PATH=1 (ablation of Algorithm 1): every node takes the fixed
# textbook step instead of the greedy choice
FIXED_PATH = os.environ.get("MJK_FIXED_PATH") == "1"


def schedule_low_pressure(order):
    """Reorder a recurrence DAG (topologically sorted node list) to keep few
    intermediates alive: greedy list scheduling that always emits the ready
    node freeing the most values (ties: original order).  Returns the new
    order and its peak number of live intermediates."""
    nodes = {id(n): n for n in order}
    users = {k: [] for k in nodes}
    for n in order:
        for d in set(id(x) for x in n.deps.values()):
            if d in nodes:
                users[d].append(id(n))
    left = {k: len(u) for k, u in users.items()}
    ndeps = {id(n): len(set(id(x) for x in n.deps.values() if id(x) in nodes)) for n in order}
    pos = {id(n): i for i, n in enumerate(order)}
    ready = [id(n) for n in order if ndeps[id(n)] == 0]
    out, live, peak = [], set(), 0
    while ready:
        best = None
        for r in ready:
            n = nodes[r]
            deps = set(id(x) for x in n.deps.values() if id(x) in nodes)
            freed = sum(1 for d in deps if left[d] == 1)
            score = (freed - (1 if left[r] > 0 else 0), -pos[r])
            if best is None or score > best[0]:
                best = (score, r)
        r = best[1]
        ready.remove(r)
        n = nodes[r]
        out.append(n)
        for d in set(id(x) for x in n.deps.values() if id(x) in nodes):
            left[d] -= 1
            if left[d] == 0:
                live.discard(d)
        if left[r] > 0:
            live.add(r)
        peak = max(peak, len(live))
        for u in users[r]:
            ndeps[u] -= 1
            if ndeps[u] == 0:
                ready.append(u)
    assert len(out) == len(order)
    return out, peak


def best_vrr(la, lb, lc, ld, targets=None):
    best = None
    for lam in ((0.0,) if FIXED_PATH else LAMBDAS):
        v = VRR(la, lb, lc, ld, lam)
        v.build(targets)
        key = (v.flops(), len(v.order))
        if best is None or key < best[0]:
            best = (key, v)
    v = best[1]
    if os.environ.get("MJK_NO_SCHED") != "1":
        v.order, v.live_peak = schedule_low_pressure(v.order)
    return v


def _axis_key(t):
    m = max(t)
    return (t.index(m), t)


def choose_passes(la, lb, lc, ld, max_acc):
    """Split the [e0|f0] targets into passes of at most max_acc accumulators.

    A pass is a group of ket components f (or bra components e) with every
    component of the other side; groups follow the dominant Cartesian axis so
    that the recurrence cones of a pass overlap as much as possible.  The
    split with the fewest total flops (the cones are recomputed per pass)
    wins.  Returns a list of target lists."""
    es = [t for l in range(la, la + lb + 1) for t in cart(l)]
    fs = [t for l in range(lc, lc + ld + 1) for t in cart(l)]
    allt = [(e, f) for e in es for f in fs]
    if len(allt) <= max_acc:
        return [allt]
    best = None
    for side in ("f", "e"):
        items, other = (fs, es) if side == "f" else (es, fs)
        per = max_acc // len(other)
        if per < 1:
            continue

        def expand(g):
            return [(e, f) for e in es for f in g] if side == "f" else [(e, f) for e in g for f in fs]

        cost = {}

        def group_flops(g):
            if g not in cost:
                cost[g] = best_vrr(la, lb, lc, ld, expand(g)).flops()
            return cost[g]

        srt = sorted(items, key=_axis_key)
        ngrp = -(-len(srt) // per)
        # balanced contiguous groups
        bounds = [round(g * len(srt) / ngrp) for g in range(ngrp + 1)]
        groups = [tuple(srt[bounds[g]:bounds[g + 1]]) for g in range(ngrp)]
        tot = sum(group_flops(g) for g in groups)
        # then a seeded local search: move one component to another group or
        # swap two, kept when the summed flops of the passes drop
        rng = random.Random((((la * 7 + lb) * 7 + lc) * 7 + ld) * 4096 + max_acc * 2 + (side == "e"))
        for _ in range(PASS_SEARCH if ngrp > 1 else 0):
            i, j = rng.sample(range(ngrp), 2)
            gi, gj = list(groups[i]), list(groups[j])
            if rng.random() < 0.5 and len(gj) < per and len(gi) > 1:
                x = rng.choice(gi)
                gi.remove(x)
                gj.append(x)
            else:
                x, y = rng.choice(gi), rng.choice(gj)
                gi[gi.index(x)] = y
                gj[gj.index(y)] = x
            ni, nj = tuple(sorted(gi, key=_axis_key)), tuple(sorted(gj, key=_axis_key))
            new = tot - group_flops(groups[i]) - group_flops(groups[j]) + group_flops(ni) + group_flops(nj)
            if new < tot:
                groups[i], groups[j], tot = ni, nj, new
        if best is None or tot < best[0]:
            best = (tot, [expand(g) for g in groups])
    if best is None:
        raise ValueError("max_acc too small for this class")
    return best[1]


# --------------------------------------------------------------------------
# HRR DAG (one side); each node is a vector over the other side's components
# --------------------------------------------------------------------------

class HRR:
    """(a, b| from [e0| with |e| in [la, la+lb]: (a,b| = (a+1_i, b-1_i| + X_i (a, b-1_i|."""

    def __init__(self, la, lb):
        self.la, self.lb = la, lb
        self.nodes = {}
        self.order = []

    def need(self, a, b):
        key = (a, b)
        if key in self.nodes:
            return self.nodes[key]
        if b == ZERO3:
            self.nodes[key] = ("base", a)
            return self.nodes[key]
        best = None
        for i in range(3):
            if b[i] == 0:
                continue
            ch = [(add(a, i), sub(b, i)), (a, sub(b, i))]
            r = sum(1 for c in ch if c in self.nodes)
            cost = (2 - r, i)
            if best is None or cost < best[0]:
                best = (cost, i, ch)
        _, i, ch = best
        self.need(*ch[0])
        self.need(*ch[1])
        node = ("hrr", a, b, i, ch[0], ch[1], len(self.order))
        self.nodes[key] = node
        self.order.append(node)
        return node

    def build(self):
        for a in cart(self.la):
            for b in cart(self.lb):
                self.need(a, b)
        return self

    def count(self):
        return len(self.order)


# --------------------------------------------------------------------------
# Code emission
# --------------------------------------------------------------------------

def cls_name(la, lb, lc, ld):
    s = "spdfgh"
    return f"{s[la]}{s[lb]}{s[lc]}{s[ld]}"


# classes whose accumulators exceed this many doubles run as several passes
MAX_ACC = int(os.environ.get("MJK_MAX_ACC", "96"))
# local-search steps over the pass groups of a split class (0: the plain
# contiguous groups)
PASS_SEARCH = int(os.environ.get("MJK_PASS_SEARCH", "400"))
# the same for the shifted classes only the nuclear gradient uses (one unit
# of angular momentum higher: more recurrence intermediates per target).
# Measured on the 60-atom gradient: 96-target passes are faster up to
# L = 7 ((dp|ds)'s kernel 1.03 -> 0.93 s), 64-target ones from L = 8 on
# ((dd|dp) 1.23 vs 1.27 s, (dd|dd) 0.70 vs 0.76 s).
GRAD_MAX_ACC = int(os.environ.get("MJK_GRAD_MAX_ACC", "64"))
GRAD_MAX_ACC_LOW_L = int(os.environ.get("MJK_GRAD_MAX_ACC_LOW_L", "96"))
GRAD_LOW_L_MAX = 7
# a compiler scheduling fence every this many recurrence nodes keeps the
# low-pressure emission order (0 = no fences)
SCHED_WINDOW = int(os.environ.get("MJK_SCHED_WINDOW", "0"))


def fence(lines, count):
    if SCHED_WINDOW and count % SCHED_WINDOW == SCHED_WINDOW - 1:
        lines.append("    __builtin_amdgcn_sched_barrier(0);")


class ClassCode:
    def __init__(self, la, lb, lc, ld, max_acc=MAX_ACC, passes=False):
        self.la, self.lb, self.lc, self.ld = la, lb, lc, ld
        self.name = cls_name(la, lb, lc, ld)
        self.vrr = best_vrr(la, lb, lc, ld)
        self.es, self.fs = self.vrr.build()
        self.eidx = {e: k for k, e in enumerate(self.es)}
        self.fidx = {f: k for k, f in enumerate(self.fs)}
        self.nacc = len(self.es) * len(self.fs)
        self.hb = HRR(la, lb).build()
        self.hk = HRR(lc, ld).build()
        nE, nF = len(self.es), len(self.fs)
        nab, ncd = ncart(la) * ncart(lb), ncart(lc) * ncart(ld)
        cost_bra_first = self.hb.count() * nF + nab * self.hk.count()
        cost_ket_first = self.hk.count() * nE + ncd * self.hb.count()
        self.bra_first = cost_bra_first <= cost_ket_first
        self.hrr_flops = 2 * min(cost_bra_first, cost_ket_first)
        self.nout = nab * ncd
        self.nab, self.ncd = nab, ncd
        self.split = self.nacc > max_acc
        self.passes = []
        # passes (and the cooperative HRR pieces) exist for split classes and,
        # on request, as a single pass for a class that fits one lane
        self.has_passes = self.split or passes
        if self.split:
            for tg in choose_passes(la, lb, lc, ld, max_acc):
                self.passes.append((tg, best_vrr(la, lb, lc, ld, tg)))
        elif passes:
            self.passes.append((list(self.vrr.built_targets), self.vrr))
        if self.has_passes:
            self.split_flops = sum(v.flops() for _, v in self.passes)
            # cooperative HRR: bra per ket column, then ket per (ab) row
            self.split_hrr_flops = 2 * (self.hb.count() * nF + nab * self.hk.count())

    # ---- VRR ----
    def emit_vrr(self):
        v = self.vrr
        L = v.L
        lines = []
        lines.append("template <typename T>")
        lines.append(f"__device__ __forceinline__ void vrr_{self.name}(const T* __restrict__ F, const VrrGeom<T>& g, "
                     f"T* __restrict__ acc)")
        lines.append("{")
        lines.append(f"    // [e0|f0]^(0) for |e| in [{self.la},{self.la + self.lb}], |f| in [{self.lc},"
                     f"{self.lc + self.ld}]; {len(v.order)} intermediates, m <= {L}")
        need_oo2p = any(n.side == "b" and "x3" in n.deps for n in v.order)
        need_oo2q = any(n.side == "k" and "x3" in n.deps for n in v.order)
        need_oo2pq = any("x5" in n.deps for n in v.order)
        targets = {}
        for e in self.es:
            for f in self.fs:
                targets[(e, f, 0)] = self.eidx[e] * len(self.fs) + self.fidx[f]
        consts = {}

        def coef(kind, k):
            key = (kind, k)
            if key not in consts:
                nm = f"c_{kind}{k}"
                base = {"p": "g.oo2p", "q": "g.oo2q", "pq": "g.oo2pq"}[kind]
                if k == 1:
                    consts[key] = base
                else:
                    consts[key] = nm
                    lines.append(f"    const T {nm} = T({k}) * {base};")
            return consts[key]

        del need_oo2p, need_oo2q, need_oo2pq
        for n in v.order:
            d = n.deps
            i = n.axis
            if n.side == "b":
                A, W, rr, kind, cnt = f"g.PA[{i}]", f"g.WP[{i}]", "g.rho_p", "p", n.e[i] - 1
                ocnt = n.f[i]
            else:
                A, W, rr, kind, cnt = f"g.QC[{i}]", f"g.WQ[{i}]", "g.rho_q", "q", n.f[i] - 1
                ocnt = n.e[i]
            expr = f"{A} * {d['x1'].name} + {W} * {d['x2'].name}"
            if "x3" in d:
                c = coef(kind, cnt)
                expr += f" + {c} * ({d['x3'].name} - {rr} * {d['x4'].name})"
            if "x5" in d:
                c = coef("pq", ocnt)
                expr += f" + {c} * {d['x5'].name}"
            key = (n.e, n.f, n.m)
            lines.append(f"    const T {n.name} = {expr};")
            if key in targets:
                lines.append(f"    acc[{targets[key]}] += {n.name};")
            fence(lines, len(lines))
        # targets that are base nodes ([00|00]^(0) for the (ss|ss) class)
        for key, k in targets.items():
            node = v.nodes[key]
            if node.side == "":
                lines.append(f"    acc[{k}] += {node.name};")
        lines.append("}")
        return "\n".join(lines)

    # ---- HRR ----
    def emit_hrr(self):
        la, lb, lc, ld = self.la, self.lb, self.lc, self.ld
        nb, nc, nd = ncart(lb), ncart(lc), ncart(ld)
        nF = len(self.fs)
        lines = []
        lines.append("template <typename T>")
        lines.append(f"__device__ __forceinline__ void hrr_{self.name}(const T* __restrict__ acc, const T AB[3], "
                     f"const T CD[3], T* __restrict__ out)")
        lines.append("{")
        hb, hk = self.hb, self.hk

        def bra_name(node_key, fk):
            node = hb.nodes[node_key]
            if node[0] == "base":
                return f"acc[{self.eidx[node[1]] * nF + fk}]"
            return f"hb{node[6]}_{fk}"

        if self.bra_first:
            # (ab|f] for every f, then the ket HRR for every (ab)
            for fk in range(nF):
                for node in hb.order:
                    _, a, b, i, c0, c1, k = node
                    lines.append(f"    const T hb{k}_{fk} = {bra_name(c0, fk)} + AB[{i}] * {bra_name(c1, fk)};")

            def abf(a, b, f):
                return bra_name((a, b), self.fidx[f])

            for a in cart(la):
                for b in cart(lb):
                    ab = cidx(a) * nb + cidx(b)
                    tag = f"{ab}"
                    names = {}

                    def kn(key):
                        node = hk.nodes[key]
                        if node[0] == "base":
                            return abf(a, b, node[1])
                        return names[key]

                    for node in hk.order:
                        _, c, d, i, c0, c1, k = node
                        nm = f"hk{k}_{tag}"
                        lines.append(f"    const T {nm} = {kn(c0)} + CD[{i}] * {kn(c1)};")
                        names[(c, d)] = nm
                    for c in cart(lc):
                        for d in cart(ld):
                            o = (ab * nc + cidx(c)) * nd + cidx(d)
                            lines.append(f"    out[{o}] = {kn((c, d))};")
        else:
            nE = len(self.es)

            def ket_name(node_key, ek):
                node = hk.nodes[node_key]
                if node[0] == "base":
                    return f"acc[{ek * nF + self.fidx[node[1]]}]"
                return f"hk{node[6]}_{ek}"

            for ek in range(nE):
                for node in hk.order:
                    _, c, d, i, c0, c1, k = node
                    lines.append(f"    const T hk{k}_{ek} = {ket_name(c0, ek)} + CD[{i}] * {ket_name(c1, ek)};")

            def ecd(e, c, d):
                return ket_name((c, d), self.eidx[e])

            for c in cart(lc):
                for d in cart(ld):
                    cd = cidx(c) * nd + cidx(d)
                    tag = f"{cd}"
                    names = {}

                    def bn(key):
                        node = hb.nodes[key]
                        if node[0] == "base":
                            return ecd(node[1], c, d)
                        return names[key]

                    for node in hb.order:
                        _, a, b, i, c0, c1, k = node
                        nm = f"hb{k}_{tag}"
                        lines.append(f"    const T {nm} = {bn(c0)} + AB[{i}] * {bn(c1)};")
                        names[(a, b)] = nm
                    for a in cart(la):
                        for b in cart(lb):
                            o = ((cidx(a) * nb + cidx(b)) * nc + cidx(c)) * nd + cidx(d)
                            lines.append(f"    out[{o}] = {bn((a, b))};")
        lines.append("}")
        return "\n".join(lines)

    # ---- split classes: VRR passes and cooperative HRR pieces ----
    def emit_vrr_pass(self, k):
        targets, v = self.passes[k]
        nF = len(self.fs)
        lines = ["template <typename T>",
                 f"__device__ __forceinline__ void vrr_{self.name}_p{k}(const T* __restrict__ F, const VrrGeom<T>& g, "
                 f"T* __restrict__ acc)", "{",
                 f"    // pass {k}: {len(targets)} of {self.nacc} targets, {len(v.order)} intermediates"]
        tmap = {(e, f, 0): j for j, (e, f) in enumerate(targets)}
        consts = {}

        def coef(kind, cnt):
            key = (kind, cnt)
            if key not in consts:
                base = {"p": "g.oo2p", "q": "g.oo2q", "pq": "g.oo2pq"}[kind]
                if cnt == 1:
                    consts[key] = base
                else:
                    consts[key] = f"c_{kind}{cnt}"
                    lines.append(f"    const T c_{kind}{cnt} = T({cnt}) * {base};")
            return consts[key]

        for n in v.order:
            d = n.deps
            i = n.axis
            if n.side == "b":
                A, W, rr, kind, cnt, ocnt = f"g.PA[{i}]", f"g.WP[{i}]", "g.rho_p", "p", n.e[i] - 1, n.f[i]
            else:
                A, W, rr, kind, cnt, ocnt = f"g.QC[{i}]", f"g.WQ[{i}]", "g.rho_q", "q", n.f[i] - 1, n.e[i]
            expr = f"{A} * {d['x1'].name} + {W} * {d['x2'].name}"
            if "x3" in d:
                expr += f" + {coef(kind, cnt)} * ({d['x3'].name} - {rr} * {d['x4'].name})"
            if "x5" in d:
                expr += f" + {coef('pq', ocnt)} * {d['x5'].name}"
            lines.append(f"    const T {n.name} = {expr};")
            key = (n.e, n.f, n.m)
            if key in tmap:
                lines.append(f"    acc[{tmap[key]}] += {n.name};")
            fence(lines, len(lines))
        for key, j in tmap.items():
            if v.nodes[key].side == "":
                lines.append(f"    acc[{j}] += {v.nodes[key].name};")
        lines.append("}")
        gmap = [self.eidx[e] * nF + self.fidx[f] for e, f in targets]
        lines.append(f"__device__ constexpr int map_{self.name}_p{k}[{len(gmap)}] = {{{', '.join(map(str, gmap))}}};")
        return "\n".join(lines)

    def emit_hrr_col_row(self):
        """hrr_bra_col: one ket column f of [e0|f0] (LDS, [e][f]) -> (ab|f] (LDS, [ab][f]);
        hrr_ket_row: one (ab) row of (ab|f] -> (ab|cd) for every cd (registers)."""
        la, lb, lc, ld = self.la, self.lb, self.lc, self.ld
        nb, nd = ncart(lb), ncart(ld)
        nF = len(self.fs)
        L = ["template <int STRIDE, typename T>",
             f"__device__ __forceinline__ void hrr_bra_col_{self.name}(const T* __restrict__ ef, int f, const T AB[3], "
             "T* __restrict__ abf)", "{",
             "    // ef holds [e0|f0] as [e][f] with element stride STRIDE"]
        hb = self.hb

        def bname(key):
            node = hb.nodes[key]
            if node[0] == "base":
                return f"ef[({self.eidx[node[1]] * nF} + f) * STRIDE]"
            return f"b{node[6]}"

        for node in hb.order:
            _, a, b, i, c0, c1, k = node
            L.append(f"    const T b{k} = {bname(c0)} + AB[{i}] * {bname(c1)};")
        for a in cart(la):
            for b in cart(lb):
                L.append(f"    abf[{(cidx(a) * nb + cidx(b)) * nF} + f] = {bname((a, b))};")
        L.append("}")
        L += ["template <typename T>",
              f"__device__ __forceinline__ void hrr_ket_row_{self.name}(const T* __restrict__ row, const T CD[3], "
              "T* __restrict__ out)", "{"]
        hk = self.hk

        def kname(key):
            node = hk.nodes[key]
            if node[0] == "base":
                return f"row[{self.fidx[node[1]]}]"
            return f"k{node[6]}"

        for node in hk.order:
            _, c, d, i, c0, c1, k = node
            L.append(f"    const T k{k} = {kname(c0)} + CD[{i}] * {kname(c1)};")
        for c in cart(lc):
            for d in cart(ld):
                L.append(f"    out[{cidx(c) * nd + cidx(d)}] = {kname((c, d))};")
        L.append("}")
        return "\n".join(L)

    def emit_split_trait(self):
        la, lb, lc, ld = self.la, self.lb, self.lc, self.ld
        P = len(self.passes)
        lines = ["template <>", f"struct EriSplit<{la}, {lb}, {lc}, {ld}> {{",
                 f"    static constexpr int NPASS = {P};",
                 f"    static constexpr int NE = {len(self.es)};", f"    static constexpr int NF = {len(self.fs)};",
                 f"    static constexpr int NACC = {self.nacc};",
                 f"    static constexpr int MAXP = {max(len(t) for t, _ in self.passes)};"]
        for k, (tg, _) in enumerate(self.passes):
            lines.append(f"    static constexpr int N{k} = {len(tg)};")
        lines.append("    template <int P> __device__ static constexpr int npass_acc() {")
        lines.append("        " + " ".join(f"if constexpr (P == {k}) return {len(tg)};" for k, (tg, _) in enumerate(self.passes))
                     + " return 0; }")
        lines.append("    template <int P> __device__ static __forceinline__ int gmap(int j) {")
        lines.append("        " + " ".join(f"if constexpr (P == {k}) return map_{self.name}_p{k}[j];"
                                           for k in range(P)) + " return 0; }")
        lines.append("    template <int P, typename T>")
        lines.append("    __device__ static __forceinline__ void vrr(const T *F, const VrrGeom<T> &g, T *acc) {")
        lines.append("        " + " ".join(f"if constexpr (P == {k}) vrr_{self.name}_p{k}<T>(F, g, acc);"
                                           for k in range(P)) + " }")
        lines.append("    template <int STRIDE, typename T>")
        lines.append("    __device__ static __forceinline__ void hrr_bra_col(const T *ef, int f, const T AB[3], T *abf)")
        lines.append(f"    {{ hrr_bra_col_{self.name}<STRIDE, T>(ef, f, AB, abf); }}")
        lines.append("    template <typename T>")
        lines.append("    __device__ static __forceinline__ void hrr_ket_row(const T *row, const T CD[3], T *out)")
        lines.append(f"    {{ hrr_ket_row_{self.name}<T>(row, CD, out); }}")
        lines.append("};")
        return "\n".join(lines)

    def info(self):
        return {
            "class": self.name, "L": self.vrr.L, "nacc": self.nacc, "nout": self.nout,
            "vrr_nodes": len(self.vrr.order), "vrr_flops": self.vrr.flops(), "vrr_lambda": self.vrr.lam,
            "hrr_flops": self.hrr_flops, "hrr_bra_first": self.bra_first,
            "split": self.split, "npass": len(self.passes) if self.split else 0,
            "split_vrr_flops": self.split_flops if self.split else None,
        }


def pair_classes(lmax):
    return [(la, lb) for la in range(lmax + 1) for lb in range(la + 1)]


def quartet_classes(lmax):
    pcs = pair_classes(lmax)
    out = []
    for X in range(len(pcs)):
        for Y in range(X + 1):
            out.append(pcs[X] + pcs[Y])
    return out


# Derivative integrals of a class, one shifted class per (centre, direction):
# d/dA_i (ab|cd) = 2 alpha (a+1_i b|cd) - a_i (a-1_i b|cd), the same on B and
# C; the fourth centre follows from translational invariance.
GRAD_KINDS = ("A+", "A-", "B+", "B-", "C+", "C-")


def grad_subclasses(la, lb, lc, ld):
    out = []
    for k, kind in enumerate(GRAD_KINDS):
        cen, up = k // 2, kind[1] == "+"
        t = [la, lb, lc, ld]
        t[cen] += 1 if up else -1
        if min(t) >= 0:
            out.append((k, tuple(t)))
    return out


def grad_digest_flops(la, lb, lc, ld, k, sub):
    """FMAs (2 flops) of contracting one shifted block with the density weights."""
    cen, up = k // 2, GRAD_KINDS[k][1] == "+"
    ls = list(sub)
    nother = 1
    for c in range(4):
        if c != cen:
            nother *= ncart(ls[c])
    ndir = sum((sum(1 for x in t if x >= 1) if up else 3) for t in cart(ls[cen]))
    return 2 * nother * ndir


HEADER = """// Generated by paper_2412_13203_amd/gen/eri_gen.py -- do not edit.
// Obara-Saika vertical and Head-Gordon-Pople horizontal recurrences of one
// angular-momentum class; path chosen by the greedy search of Section 6.
#pragma once
"""


def emit_trait(cc, full):
    la, lb, lc, ld = cc.la, cc.lb, cc.lc, cc.ld
    lines = [
        "template <>",
        f"struct EriClass<{la}, {lb}, {lc}, {ld}> {{",
        f"    static constexpr int NACC = {cc.nacc};",
        f"    static constexpr int NOUT = {cc.nout};",
        f"    static constexpr bool SPLIT = {'true' if cc.split else 'false'};",
    ]
    if full:
        lines += [
            "    template <typename T>",
            "    __device__ static __forceinline__ void vrr(const T *F, const VrrGeom<T> &g, T *acc)",
            f"    {{ vrr_{cc.name}<T>(F, g, acc); }}",
            "    template <typename T>",
            "    __device__ static __forceinline__ void hrr(const T *acc, const T AB[3], const T CD[3], T *out)",
            f"    {{ hrr_{cc.name}<T>(acc, AB, CD, out); }}",
        ]
    lines.append("};")
    return "\n".join(lines)


def _write(path, text):
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        fh.write(text)
    os.replace(tmp, path)


def _class_job(args):
    """Emit one class header; returns its name, text and counts."""
    (la, lb, lc, ld), (fwd, grad) = args
    gmax = GRAD_MAX_ACC_LOW_L if la + lb + lc + ld <= GRAD_LOW_L_MAX else GRAD_MAX_ACC
    cc = ClassCode(la, lb, lc, ld, max_acc=MAX_ACC if fwd else gmax, passes=grad)
    # single-pass code only where one lane holds the class: split classes run
    # J/K, eri_class and Schwarz through their passes and the cooperative HRR
    full = not cc.split
    body = [HEADER]
    if full:
        body.append(cc.emit_vrr())
        body.append(cc.emit_hrr())
    body.append(emit_trait(cc, full))
    if cc.has_passes:
        for k in range(len(cc.passes)):
            body.append(cc.emit_vrr_pass(k))
        body.append(cc.emit_hrr_col_row())
        body.append(cc.emit_split_trait())
    info = cc.info()
    info["forward"] = fwd
    return cc.name, "\n\n".join(body) + "\n", info


def generate(outdir, lmax=2, jobs=None, grad_lmax=2):
    """Write one header per class (cls_<name>.inc), one translation unit per
    J/K class and per gradient class, and dispatch.inc.  The nuclear gradient
    covers the classes with every l <= grad_lmax (its shifted classes reach
    grad_lmax + 1)."""
    os.makedirs(outdir, exist_ok=True)
    fwd = quartet_classes(lmax)
    grad_lmax = min(grad_lmax, lmax)
    has_grad = lambda c: max(c) <= grad_lmax  # noqa: E731
    need = {c: [True, False] for c in fwd}  # (J/K class, shifted class of a gradient)
    for c in fwd:
        if not has_grad(c):
            continue
        for _, t in grad_subclasses(*c):
            need.setdefault(t, [False, False])[1] = True
    work = sorted(need.items(), key=lambda kv: -sum(kv[0]))
    jobs = jobs or min(8, os.cpu_count() or 1)
    if jobs > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(jobs) as pool:
            res = pool.map(_class_job, work, chunksize=1)
    else:
        res = [_class_job(w) for w in work]
    infos = {}
    for (t, _), (name, text, info) in zip(work, res):
        _write(os.path.join(outdir, f"cls_{name}.inc"), text)
        infos[t] = info
    tus = []
    for c in fwd:
        name = cls_name(*c)
        split = infos[c]["split"]
        head = ["// Generated by paper_2412_13203_amd/gen/eri_gen.py -- do not edit.",
                '#include "../kernels.hpp"', "namespace mjk {", f'#include "cls_{name}.inc"']
        units = []
        if split:
            # J/K and eri_class/Schwarz kernels of a split class in two units
            units.append(("", [f"MJK_DEFINE_CLASS_SPLIT_JK({c[0]}, {c[1]}, {c[2]}, {c[3]}, {name})"]))
            units.append(("eri_", [f"MJK_DEFINE_CLASS_SPLIT_ERI({c[0]}, {c[1]}, {c[2]}, {c[3]}, {name})"]))
        else:
            body = [f"MJK_DEFINE_CLASS({c[0]}, {c[1]}, {c[2]}, {c[3]}, {name})"]
            if c[:2] == c[2:]:
                body.append(f"MJK_DEFINE_SCHWARZ({c[0]}, {c[1]}, {name[:2]})")
            units.append(("", body))
        for prefix, body in units:
            path = os.path.join(outdir, f"tu_{prefix}{name}.hip")
            _write(path, "\n".join(head + body + ["}  // namespace mjk"]) + "\n")
            tus.append(path)
        if not has_grad(c):
            continue
        lines = ["// Generated by paper_2412_13203_amd/gen/eri_gen.py -- do not edit.",
                 '#include "../kernels.hpp"', '#include "../grad_kernels.hpp"', "namespace mjk {"]
        for _, t in grad_subclasses(*c):
            lines.append(f'#include "cls_{cls_name(*t)}.inc"')
        lines.append(f"MJK_DEFINE_GRAD({c[0]}, {c[1]}, {c[2]}, {c[3]}, {name})")
        lines.append("}  // namespace mjk")
        path = os.path.join(outdir, f"tu_grad_{name}.hip")
        _write(path, "\n".join(lines) + "\n")
        tus.append(path)
    # dispatch table, indexed by quartet class X(X+1)/2 + Y over pair classes
    d = ["// Generated by paper_2412_13203_amd/gen/eri_gen.py -- do not edit.", "#pragma once",
         '#include "../mjk_types.hpp"', "namespace mjk {"]
    for c in fwd:
        name = cls_name(*c)
        d.append(f"int launch_jk_{name}(const JKLaunch &, hipStream_t);")
        d.append(f"int launch_jk32_{name}(const JKLaunch &, hipStream_t);")
        d.append(f"int launch_eri_{name}(const EriLaunch &, hipStream_t);")
        d.append(f"int launch_eri32_{name}(const EriLaunch &, hipStream_t);")
        if has_grad(c):
            d.append(f"int launch_grad_{name}(const JKLaunch &, hipStream_t);")
            d.append(f"size_t grad_stage_nacc_{name}();")
        if c[:2] == c[2:] and not infos[c]["split"]:
            d.append(f"int launch_schwarz_{name[:2]}(const SchwarzLaunch &, hipStream_t);")
    d.append(f"constexpr int kLmax = {lmax};")
    d.append(f"constexpr int kGradLmax = {grad_lmax};")
    d.append(f"constexpr int kNumPairClasses = {len(pair_classes(lmax))};")
    d.append(f"constexpr int kNumQuartetClasses = {len(fwd)};")
    d.append("static const ClassEntry kClassTable[kNumQuartetClasses] = {")
    for c in fwd:
        name = cls_name(*c)
        cc = infos[c]
        # split diagonal classes compute Schwarz factors through their eri launcher
        sch = f"launch_schwarz_{name[:2]}" if c[:2] == c[2:] and not cc["split"] else "nullptr"
        # algorithmic work: the single-pass recurrence and the cheaper HRR order,
        # whatever the kernel executes (passes recompute shared intermediates)
        subs = grad_subclasses(*c) if has_grad(c) else []
        g_vrr = sum(infos[t]["vrr_flops"] + 1 for _, t in subs)  # +1: the weight
        g_up = sum(1 for k, _ in subs if GRAD_KINDS[k][1] == "+")
        g_dn = len(subs) - g_up
        nw = ncart(c[0]) * ncart(c[1]) * ncart(c[2]) * ncart(c[3])
        g_q = (sum(infos[t]["hrr_flops"] + grad_digest_flops(*c, k, t) for k, t in subs) + 6 * nw) if subs else 0
        gl = f"launch_grad_{name}, grad_stage_nacc_{name}" if has_grad(c) else "nullptr, nullptr"
        d.append(f"    {{{c[0]}, {c[1]}, {c[2]}, {c[3]}, {cc['nacc']}, {cc['nout']}, {cc['vrr_flops']}, "
                 f"{cc['hrr_flops']}, {int(cc['split'])}, {cc['npass']}, launch_jk_{name}, launch_jk32_{name}, "
                 f"launch_eri_{name}, launch_eri32_{name}, {sch}, {gl}, {g_vrr}, {g_up}, {g_dn}, "
                 f"{g_q}}},")
    d.append("};")
    d.append("}  // namespace mjk")
    _write(os.path.join(outdir, "dispatch.inc"), "\n".join(d) + "\n")
    with open(os.path.join(outdir, "opcount.json"), "w") as fh:
        json.dump([dict(v, tuple=list(k)) for k, v in sorted(infos.items())], fh, indent=1)
    return infos, tus


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else "gen_out"
    lmax = int(sys.argv[2]) if len(sys.argv) > 2 else 2
    infos, tus = generate(out, lmax)
    for k, i in sorted(infos.items()):
        print(k, i)
