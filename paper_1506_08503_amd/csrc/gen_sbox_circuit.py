"""Generate the bitsliced AES S-box circuit (sbox_circuit.inc) from field arithmetic.

    python paper_1506_08503_amd/csrc/gen_sbox_circuit.py

SubBytes is inversion in GF(2^8) followed by an affine map over GF(2) (the
paper's App. A2).  Bitsliced, every bit of a byte is a 32-bit word holding that
bit for 32 blocks, so the S-box must be a circuit of XOR / AND gates.  Inversion
is cheap as a circuit in a tower field GF(((2^2)^2)^2):

  GF(4)   = GF(2)[W]/(W^2 + W + 1)
  GF(16)  = GF(4)[Z]/(Z^2 + Z + N),   N in GF(4)  with trace 1
  GF(256) = GF(16)[Y]/(Y^2 + Y + M),  M in GF(16) with trace 1

  (a1 Y + a0)^-1 = (a1 / d) Y + (a0 + a1) / d,  d = M a1^2 + a1 a0 + a0^2
  (d1 Z + d0)^-1 = (d1 / e) Z + (d0 + d1) / e,  e = N d1^2 + d1 d0 + d0^2
  e^-1 = e^2 in GF(4).

The AES field (polynomial 0x11B, sec. II) maps onto the tower by x -> beta,
beta a root of x^8 + x^4 + x^3 + x + 1 in the tower; the map and the affine
transform become 8 x 8 GF(2) matrices at the input and output.  Linear layers
are built with greedy common-subexpression elimination (pairs shared by most
outputs first).  Every (N, M, beta) choice is tried.

gfx950 has a three-input logic op (v_bitop3_b32, any function of three
words), so the gate graph is then covered by three-input operations: every
gate gets its 3-feasible cuts (sets of at most three wires that separate it
from the inputs), and an integer program picks the cuts that implement all
outputs with the fewest operations (an operation needs every gate among its
cut leaves to be implemented too).  The program runs (HiGHS through
scipy.optimize.milp, with a node limit so that the result is reproducible) on
the few circuits whose greedy single-fanout folding is smallest, and the
smallest cover is kept.  The affine constant 0x63 is NOT part of the circuit: it passes through
MixColumns unchanged (2 + 3 + 1 + 1 = 1 in GF(2^8)), so the kernels fold it into
the round keys of rounds 1..Nr.

The script checks the circuit against the S-box on all 256 inputs before it
writes anything.
"""
from __future__ import annotations

import itertools
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "sbox_circuit.inc")


# ------------------------------------------------------------ field arithmetic
def gf4_mul(a, b):
    # a = a1 W + a0, W^2 = W + 1
    a1, a0, b1, b0 = a >> 1, a & 1, b >> 1, b & 1
    hi = (a1 & b1) ^ (a1 & b0) ^ (a0 & b1)
    lo = (a1 & b1) ^ (a0 & b0)
    return (hi << 1) | lo


def gf16_mul(a, b, n):
    a1, a0, b1, b0 = a >> 2, a & 3, b >> 2, b & 3
    p = gf4_mul(a1, b1)
    hi = p ^ gf4_mul(a1, b0) ^ gf4_mul(a0, b1)
    lo = gf4_mul(n, p) ^ gf4_mul(a0, b0)
    return (hi << 2) | lo


def gf256t_mul(a, b, n, m):
    a1, a0, b1, b0 = a >> 4, a & 15, b >> 4, b & 15
    p = gf16_mul(a1, b1, n)
    hi = p ^ gf16_mul(a1, b0, n) ^ gf16_mul(a0, b1, n)
    lo = gf16_mul(m, p, n) ^ gf16_mul(a0, b0, n)
    return (hi << 4) | lo


def aes_mul(a, b):
    r = 0
    while b:
        if b & 1:
            r ^= a
        a <<= 1
        if a & 0x100:
            a ^= 0x11B
        b >>= 1
    return r


def aes_sbox():
    inv = [0] * 256
    for a in range(1, 256):
        for b in range(1, 256):
            if aes_mul(a, b) == 1:
                inv[a] = b
                break
    out = []
    for x in range(256):
        v = inv[x]
        s = v
        for k in range(1, 5):
            s ^= ((v << k) | (v >> (8 - k))) & 0xFF
        out.append(s ^ 0x63)
    return out


def trace(x, mul, deg):
    t, p = 0, x
    for _ in range(deg):
        t ^= p
        p = mul(p, p)
    return t


# --------------------------------------------------------------- GF(2) matrices
def mat_apply(rows, v):
    """rows[i] is a bitmask over input bits; returns output bits as an int."""
    out = 0
    for i, r in enumerate(rows):
        out |= (bin(r & v).count("1") & 1) << i
    return out


def mat_from_fn(fn):
    cols = [fn(1 << k) for k in range(8)]
    rows = []
    for i in range(8):
        r = 0
        for k in range(8):
            if (cols[k] >> i) & 1:
                r |= 1 << k
        rows.append(r)
    return rows


def mat_inverse(rows):
    n = 8
    a = [(rows[i], 1 << i) for i in range(n)]
    for c in range(n):
        piv = next((i for i in range(c, n) if (a[i][0] >> c) & 1), None)
        if piv is None:
            return None
        a[c], a[piv] = a[piv], a[c]
        for i in range(n):
            if i != c and (a[i][0] >> c) & 1:
                a[i] = (a[i][0] ^ a[c][0], a[i][1] ^ a[c][1])
    return [a[i][1] for i in range(n)]


# ------------------------------------------------------------------- circuit
class Circuit:
    """Gates over named wires; wire values are 'x0'..'x7' inputs or t<k>."""

    def __init__(self, rng=None):
        self.gates = []      # (dst, op, a, b)
        self.n = 0
        self.cache = {}
        self.rng = rng       # random tie-breaking in linear() when given

    def new(self, op, a, b):
        key = (op, min(a, b), max(a, b))
        if key in self.cache:
            return self.cache[key]
        w = "t%d" % self.n
        self.n += 1
        self.gates.append((w, op, a, b))
        self.cache[key] = w
        return w

    def xor(self, a, b):
        if a is None:
            return b
        if b is None:
            return a
        return self.new("^", a, b)

    def and_(self, a, b):
        if a is None or b is None:
            return None
        return self.new("&", a, b)

    def linear(self, targets, basis):
        """XOR-combinations of basis wires: targets are bitmasks over `basis`.
        Greedy pairing (most shared pair first)."""
        basis = list(basis)
        rows = [t for t in targets]
        wires = list(basis)
        while True:
            counts = {}
            for r in rows:
                bits = [i for i in range(len(wires)) if (r >> i) & 1]
                if len(bits) < 2:
                    continue
                for p in itertools.combinations(bits, 2):
                    counts[p] = counts.get(p, 0) + 1
            if not counts:
                break
            top = max(counts.values())
            best = sorted(p for p, v in counts.items() if v == top)
            (i, j) = best[self.rng.randrange(len(best))] if self.rng else best[0]
            w = self.xor(wires[i], wires[j])
            wires.append(w)
            k = len(wires) - 1
            new_rows = []
            for r in rows:
                if (r >> i) & 1 and (r >> j) & 1:
                    r ^= (1 << i) | (1 << j)
                    r |= 1 << k
                new_rows.append(r)
            rows = new_rows
        out = []
        for r in rows:
            bits = [i for i in range(len(wires)) if (r >> i) & 1]
            out.append(wires[bits[0]] if bits else None)
        return out


def affine_lin(v):
    """App. A2 affine map without its constant: v ^ rotl(v,1..4)."""
    s = v
    for k in range(1, 5):
        s ^= ((v << k) | (v >> (8 - k))) & 0xFF
    return s


def build(n, m, beta, inverse=False, rng=None):
    """Circuit for one (N, M, beta) choice computing
         forward:  L(inv(x))       = S(x) ^ 0x63
         inverse:  inv(L^-1(y))    = S^-1(y ^ 0x63)
    where L is the linear part of the affine map."""
    mul = lambda a, b: gf256t_mul(a, b, n, m)
    # input map: AES bits -> tower bits
    def to_tower(v):
        r, p = 0, 1
        for k in range(8):
            if (v >> k) & 1:
                r ^= p
            p = mul(p, beta)
        return r
    X = mat_from_fn(to_tower)
    Xinv = mat_inverse(X)
    if Xinv is None:
        return None
    if inverse:
        Linv = mat_inverse(mat_from_fn(affine_lin))
        # input: undo the affine map, then into the tower; output: back to AES bits
        X = mat_from_fn(lambda v: mat_apply(X, mat_apply(Linv, v)))
        Yrows = Xinv
    else:
        # output map: tower bits -> AES bits -> affine (without the constant)
        Yrows = mat_from_fn(lambda v: affine_lin(mat_apply(Xinv, v)))

    c = Circuit(rng)
    xin = ["x%d" % i for i in range(8)]

    # Tower bits of the input as linear forms over the 8 input bits; all the
    # GF(4)-level sums the multipliers need are linear forms too.
    a_bits = X  # a_bits[i] = bitmask over x of tower bit i
    # bit layout of an element of GF(256)t: [a0(4 bits: h0(2) h1(2)), a1(4 bits)]

    def lin_sum(*forms):
        r = 0
        for f in forms:
            r ^= f
        return r

    # --- GF(4)/GF(16) symbolic helpers over "forms" (bitmask over inputs) ---
    # For the top layer we express every needed operand as a linear form of x.
    a0 = [a_bits[0], a_bits[1], a_bits[2], a_bits[3]]
    a1 = [a_bits[4], a_bits[5], a_bits[6], a_bits[7]]

    def sq16_form(h):
        # squaring in GF(16) is linear: compute matrix on 4-bit values
        def f(v):
            return gf16_mul(v, v, n)
        return [lin_sum(*[h[k] for k in range(4) if (f(1 << k) >> i) & 1]) for i in range(4)]

    def scale16_form(h, cst):
        def f(v):
            return gf16_mul(cst, v, n)
        return [lin_sum(*[h[k] for k in range(4) if (f(1 << k) >> i) & 1]) for i in range(4)]

    # d = M a1^2 + a0^2 + a1*a0; the product a1*a0 is nonlinear: Karatsuba over GF(4)
    lin_part = [x ^ y for x, y in zip(scale16_form(sq16_form(a1), m), sq16_form(a0))]

    # operands of a1*a0 (GF(16) Karatsuba) at GF(4) level, then GF(4) Karatsuba:
    def gf16_operands(h, g):
        h1, h0 = h[2:4], h[0:2]
        g1, g0 = g[2:4], g[0:2]
        hs = [h1[0] ^ h0[0], h1[1] ^ h0[1]]
        gs = [g1[0] ^ g0[0], g1[1] ^ g0[1]]
        pairs = [(h1, g1), (h0, g0), (hs, gs)]
        ops = []
        for u, v in pairs:
            # GF(4) Karatsuba products: u1v1, u0v0, (u1+u0)(v1+v0)
            ops.append([(u[1], v[1]), (u[0], v[0]), (u[1] ^ u[0], v[1] ^ v[0])])
        return ops

    # All linear forms needed at the top: operands of a1*a0 products, lin_part,
    # and operands of the final products a1*dinv, (a0+a1)*dinv (their x-side).
    prod1 = gf16_operands(a1, a0)
    a01 = [x ^ y for x, y in zip(a0, a1)]

    def gf4_split(h):
        # operands needed when h (4 forms) multiplies an unknown GF(16) value:
        h1, h0 = h[2:4], h[0:2]
        hs = [h1[0] ^ h0[0], h1[1] ^ h0[1]]
        out = []
        for u in (h1, h0, hs):
            out += [u[1], u[0], u[1] ^ u[0]]
        return out

    top_forms = []
    for grp in prod1:
        for u, v in grp:
            top_forms += [u, v]
    top_forms += lin_part
    top_forms += gf4_split(a1) + gf4_split(a01)
    uniq = []
    for f in top_forms:
        if f and f not in uniq:
            uniq.append(f)
    # single-bit forms are the inputs themselves
    wires = c.linear(uniq, xin)
    form_wire = dict(zip(uniq, wires))

    def W(form):
        return form_wire[form] if form else None

    # --- nonlinear core ---
    def gf4_mul_w(u1, u0, v1, v0, us=None, vs=None):
        """Karatsuba GF(4) product of wire pairs (hi, lo); returns (hi, lo)."""
        p11 = c.and_(u1, v1)
        p00 = c.and_(u0, v0)
        us = us if us is not None else c.xor(u1, u0)
        vs = vs if vs is not None else c.xor(v1, v0)
        pss = c.and_(us, vs)
        hi = c.xor(pss, p00)
        lo = c.xor(p11, p00)
        return hi, lo

    def gf4_mul_const(u1, u0, cst):
        # multiplication by a GF(4) constant is linear on (u1, u0)
        r = gf4_mul(cst, 2), gf4_mul(cst, 1)  # images of W and 1
        hi = lo = None
        for bitw, img in ((u1, r[0]), (u0, r[1])):
            if img >> 1 & 1:
                hi = c.xor(hi, bitw)
            if img & 1:
                lo = c.xor(lo, bitw)
        return hi, lo

    # a1 * a0 in GF(16) with top-layer operands
    def gf16_mul_top(grp):
        # grp: three GF(4) products (h1g1, h0g0, hsgs), each with 3 AND operand pairs
        res = []
        for trip in grp:
            (u11, v11), (u00, v00), (uss, vss) = trip
            p11 = c.and_(W(u11), W(v11))
            p00 = c.and_(W(u00), W(v00))
            pss = c.and_(W(uss), W(vss))
            res.append((c.xor(pss, p00), c.xor(p11, p00)))
        (p1h, p1l), (q1h, q1l), (r1h, r1l) = res   # p = h1g1, q = h0g0, r = (h1+h0)(g1+g0)
        # Z coeff = r + q ; const = N p + q
        zh, zl = c.xor(r1h, q1h), c.xor(r1l, q1l)
        nph, npl = gf4_mul_const(p1h, p1l, n)
        ch, cl = c.xor(nph, q1h), c.xor(npl, q1l)
        return [cl, ch, zl, zh]   # [lo-lo, lo-hi, hi-lo, hi-hi] bit order of GF(16)

    prod = gf16_mul_top(prod1)
    d = [c.xor(prod[i], W(lin_part[i])) if lin_part[i] else prod[i] for i in range(4)]
    # d = d1 Z + d0 in GF(16); inverse via GF(4)
    d0l, d0h, d1l, d1h = d
    # e = N d1^2 + d1 d0 + d0^2
    def sq4(h, l):
        # (h W + l)^2 = h W + (h + l)
        return h, c.xor(h, l)
    s1h, s1l = sq4(d1h, d1l)
    nsh, nsl = gf4_mul_const(s1h, s1l, n)
    s0h, s0l = sq4(d0h, d0l)
    mh, ml = gf4_mul_w(d1h, d1l, d0h, d0l)
    eh = c.xor(c.xor(nsh, s0h), mh)
    el = c.xor(c.xor(nsl, s0l), ml)
    ih, il = sq4(eh, el)                       # e^-1 = e^2 in GF(4)
    ish = c.xor(ih, il)
    o1h, o1l = gf4_mul_w(d1h, d1l, ih, il, vs=ish)
    dsh, dsl = c.xor(d1h, d0h), c.xor(d1l, d0l)
    o0h, o0l = gf4_mul_w(dsh, dsl, ih, il, vs=ish)
    dinv = [o0l, o0h, o1l, o1h]

    # final products a1 * dinv and (a0 + a1) * dinv: x-side operands are top forms
    def gf16_mul_xw(h, gw):
        h1, h0 = h[2:4], h[0:2]
        hs = [h1[0] ^ h0[0], h1[1] ^ h0[1]]
        g0l, g0h, g1l, g1h = gw
        gsl, gsh = c.xor(g1l, g0l), c.xor(g1h, g0h)
        res = []
        for u, (vh, vl) in ((h1, (g1h, g1l)), (h0, (g0h, g0l)), (hs, (gsh, gsl))):
            p11 = c.and_(W(u[1]), vh)
            p00 = c.and_(W(u[0]), vl)
            pss = c.and_(W(u[1] ^ u[0]), c.xor(vh, vl))
            res.append((c.xor(pss, p00), c.xor(p11, p00)))
        (p1h, p1l), (q1h, q1l), (r1h, r1l) = res
        zh, zl = c.xor(r1h, q1h), c.xor(r1l, q1l)
        nph, npl = gf4_mul_const(p1h, p1l, n)
        ch, cl = c.xor(nph, q1h), c.xor(npl, q1l)
        return [cl, ch, zl, zh]

    out1 = gf16_mul_xw(a1, dinv)
    out0 = gf16_mul_xw(a01, dinv)
    inv_bits = out0 + out1      # tower bits 0..7 of the inverse

    # bottom layer: out_i = XOR of inv_bits selected by Yrows[i]
    outs = c.linear(Yrows, inv_bits)
    return c, outs


# --------------------------------------------------------------- gate fusion
# gfx950's v_bitop3_b32 computes any boolean function of three 32-bit
# operands: result bit = bit (4 a + 2 b + c) of an 8-bit table.  A gate whose
# only use is another gate can be folded into that gate when the pair reads at
# most three distinct wires.
TT_A, TT_B, TT_C = 0xF0, 0xCC, 0xAA


def fuse(c, outs):
    """Returns fused ops [(dst, leaves(list of 1..3 wires), expr)] in order,
    where expr is a nested tuple over the leaves; inlined gates disappear."""
    gates = {dst: (op, a, b) for dst, op, a, b in c.gates}
    uses = {}
    for dst, op, a, b in c.gates:
        for w in (a, b):
            uses[w] = uses.get(w, 0) + 1
    for o in outs:
        uses[o] = uses.get(o, 0) + 1
    inlined = set()
    exprs = {}

    def leaves_of(e, acc):
        if isinstance(e, str):
            if e not in acc:
                acc.append(e)
        else:
            leaves_of(e[1], acc)
            leaves_of(e[2], acc)
        return acc

    order = [dst for dst, _, _, _ in c.gates]
    for dst in order:
        op, a, b = gates[dst]
        e = (op, a, b)
        for side in (1, 2):
            child = e[side]
            if child in gates and uses.get(child, 0) == 1 and child not in outs:
                cand = list(e)
                cand[side] = exprs[child]
                cand = tuple(cand)
                if len(leaves_of(cand, [])) <= 3:
                    e = cand
                    inlined.add(child)
        exprs[dst] = e
    fused = []
    for dst in order:
        if dst in inlined:
            continue
        e = exprs[dst]
        fused.append((dst, leaves_of(e, []), e))
    return fused


def lut3_cover(c, outs, node_limit=2000):
    """Cover the gate graph with three-input operations; returns the same
    [(dst, leaves, expr)] list as fuse(), or None if no cover was found."""
    import numpy as np
    from scipy.optimize import Bounds, LinearConstraint, milp
    from scipy.sparse import coo_matrix
    gates = {dst: (op, a, b) for dst, op, a, b in c.gates}
    order = [dst for dst, _, _, _ in c.gates]
    cuts = {}

    def with_trivial(w):
        return cuts[w] + [frozenset([w])] if w in gates else [frozenset([w])]
    for dst in order:
        _, a, b = gates[dst]
        found = {ca | cb for ca in with_trivial(a) for cb in with_trivial(b)
                 if len(ca | cb) <= 3}
        keep = []
        for cut in sorted(found, key=lambda k: (len(k), sorted(k))):
            if not any(k <= cut for k in keep):
                keep.append(cut)
        cuts[dst] = keep
    var = [(dst, cut) for dst in order for cut in cuts[dst]]
    index = {v: i for i, v in enumerate(var)}
    rows, cols, vals, lo, hi = [], [], [], [], []

    def constraint(coef, low, high):
        for j, v in coef.items():
            rows.append(len(lo))
            cols.append(j)
            vals.append(v)
        lo.append(low)
        hi.append(high)
    for o in sorted(set(outs)):
        if o in gates:
            constraint({index[(o, cut)]: 1 for cut in cuts[o]}, 1, 1)
    for dst in order:
        constraint({index[(dst, cut)]: 1 for cut in cuts[dst]}, 0, 1)
    for (dst, cut), i in index.items():
        for leaf in sorted(cut):
            if leaf in gates:
                coef = {index[(leaf, k)]: 1 for k in cuts[leaf]}
                coef[i] = coef.get(i, 0) - 1
                constraint(coef, 0, np.inf)
    a = coo_matrix((vals, (rows, cols)), shape=(len(lo), len(var))).tocsr()
    res = milp(c=np.ones(len(var)), constraints=LinearConstraint(a, np.array(lo), np.array(hi)),
               integrality=np.ones(len(var)), bounds=Bounds(0, 1),
               options={"node_limit": node_limit, "disp": False})
    if res.x is None:
        return None
    chosen = {var[i][0]: var[i][1] for i, v in enumerate(res.x) if v > 0.5}

    def expr(w, cut):
        if w in cut or w not in gates:
            return w
        op, x, y = gates[w]
        return (op, expr(x, cut), expr(y, cut))

    def leaves_of(e, acc):
        if isinstance(e, str):
            if e not in acc:
                acc.append(e)
        else:
            leaves_of(e[1], acc)
            leaves_of(e[2], acc)
        return acc
    out = []
    for dst in order:
        if dst in chosen:
            e = expr(dst, chosen[dst])
            out.append((dst, leaves_of(e, []), e))
    return out


def eval_expr(e, env):
    if isinstance(e, str):
        return env[e]
    op, a, b = e
    va, vb = eval_expr(a, env), eval_expr(b, env)
    return va ^ vb if op == "^" else va & vb


def truth_table(e, leaves):
    """8-bit table of e with leaves[0..2] as the three bitop3 operands."""
    env = dict(zip(leaves, (TT_A, TT_B, TT_C)))
    return eval_expr(e, env) & 0xFF


def evaluate_fused(fused, outs, x):
    """Evaluate the fused op list with bitop3 semantics (bit-serial, one input)."""
    val = {"x%d" % i: (x >> i) & 1 for i in range(8)}
    for dst, leaves, e in fused:
        tt = truth_table(e, leaves)
        bits = [val[w] for w in leaves] + [0] * (3 - len(leaves))
        val[dst] = (tt >> (4 * bits[0] + 2 * bits[1] + bits[2])) & 1
    return sum(val[o] << i for i, o in enumerate(outs))


def evaluate(c, outs, x):
    val = {"x%d" % i: (x >> i) & 1 for i in range(8)}
    for dst, op, a, b in c.gates:
        va, vb = val[a], val[b]
        val[dst] = va ^ vb if op == "^" else va & vb
    return sum(val[o] << i for i, o in enumerate(outs))


def search(target, inverse, trials=1, ilp_candidates=4):
    """All (N, M, beta) towers (and `trials` randomized linear layers each);
    the circuits with the smallest greedy folding are covered exactly and the
    smallest result is returned."""
    import random
    cands = []
    for n in (2, 3):                     # W, W^2 (trace 1 in GF(4))
        if trace(n, gf4_mul, 2) != 1:
            continue
        for m in range(1, 16):
            if trace(m, lambda a, b: gf16_mul(a, b, n), 4) != 1:
                continue
            mul = lambda a, b, n=n, m=m: gf256t_mul(a, b, n, m)
            for beta in range(2, 256):
                # beta^8 + beta^4 + beta^3 + beta + 1 == 0
                pw = [1]
                for _ in range(8):
                    pw.append(mul(pw[-1], beta))
                if pw[8] ^ pw[4] ^ pw[3] ^ pw[1] ^ pw[0]:
                    continue
                for trial in range(trials):
                    rng = random.Random(trial * 7919 + beta) if trial else None
                    res = build(n, m, beta, inverse, rng)
                    if res is None:
                        break
                    cands.append(check(res, target, n, m, beta))
    cands.sort(key=lambda b: (b[0], b[7]))
    best = cands[0]
    for cand in cands[:ilp_candidates]:
        c, outs = cand[8]
        cover = lut3_cover(c, outs)
        if cover is None:
            continue
        if any(evaluate_fused(cover, outs, x) != target[x] for x in range(256)):
            raise SystemExit("three-input cover mismatch")
        if len(cover) < best[0]:
            best = (len(cover),) + cand[1:5] + (cover,) + cand[6:]
    return best


def check(res, target, n, m, beta):
    """Check one candidate circuit on all 256 inputs (plain and greedily
    folded) and return its record."""
    c, outs = res
    if any(evaluate(c, outs, x) != target[x] for x in range(256)):
        raise SystemExit("circuit mismatch for N=%d M=%d beta=%d" % (n, m, beta))
    fused = fuse(c, outs)
    if any(evaluate_fused(fused, outs, x) != target[x] for x in range(256)):
        raise SystemExit("fused circuit mismatch for N=%d M=%d beta=%d" % (n, m, beta))
    nand = sum(1 for g in c.gates if g[1] == "&")
    return (len(fused), nand, n, m, beta, fused, outs, len(c.gates), res)


def emit(name, what, best):
    nops, nand, n, m, beta, fused, outs, ngates = best[:8]
    lines = ["// %s: tower field GF(((2^2)^2)^2), N=%d M=%d beta=0x%02x;"
             % (what, n, m, beta),
             "// %d gates (%d AND) covered by %d VALU ops (two-input XOR/AND or one"
             % (ngates, nand, nops),
             "// three-input v_bitop3_b32 each).  Checked on all 256 inputs by the generator.",
             "#define %s(x0, x1, x2, x3, x4, x5, x6, x7, y0, y1, y2, y3, y4, y5, y6, y7) \\"
             % name,
             "    do { \\"]
    for dst, leaves, e in fused:
        if isinstance(e[1], str) and isinstance(e[2], str):
            rhs = "%s %s %s" % (e[1], e[0], e[2])
        else:
            ops = leaves + ["0u"] * (3 - len(leaves))
            rhs = "__builtin_amdgcn_bitop3_b32(%s, %s, %s, 0x%02x)" % (
                ops[0], ops[1], ops[2], truth_table(e, leaves))
        lines.append("        const uint32_t %s = %s; \\" % (dst, rhs))
    for i, o in enumerate(outs):
        lines.append("        y%d = %s; \\" % (i, o))
    lines.append("    } while (0)")
    return lines


def main():
    sbox = aes_sbox()
    inv_sbox = [0] * 256
    for x, y in enumerate(sbox):
        inv_sbox[y] = x
    trials = int(os.environ.get("SBOX_SEARCH_TRIALS", "6"))
    ilp = int(os.environ.get("SBOX_ILP_CANDIDATES", "4"))
    fwd = search([sbox[x] ^ 0x63 for x in range(256)], False, trials, ilp)
    inv = search([inv_sbox[y ^ 0x63] for y in range(256)], True, trials, ilp)
    lines = ["// Generated by gen_sbox_circuit.py -- do not edit.",
             "// Bitsliced AES S-boxes with the affine constant 0x63 left out (the",
             "// kernels fold it into the round keys).  Inputs x0..x7 and outputs",
             "// y0..y7 are the bits of a byte, least significant first.", ""]
    lines += emit("AESMI_SBOX_CIRCUIT", "S(x) ^ 0x63", fwd) + [""]
    lines += emit("AESMI_INV_SBOX_CIRCUIT", "S^-1(y ^ 0x63)", inv)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    for tag, b in (("forward", fwd), ("inverse", inv)):
        print("%s: %d ops from %d gates (%d AND), N=%d M=%d beta=0x%02x"
              % (tag, b[0], b[7], b[1], b[2], b[3], b[4]))


if __name__ == "__main__":
    main()
