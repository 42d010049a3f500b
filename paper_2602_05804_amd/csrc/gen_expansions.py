#!/usr/bin/env python3
"""Emit expansions_gen.h: straight-line Cartesian expansion code for p = 0..4.

Build step of the HIP library (run by the package build; the output is also
committed).  For each order P it writes a specialisation of
``sfmm::Exp<P>`` with these device functions, fully unrolled so every
coefficient lives in a register:

  p2m_add  Q_a += m b^a / a!                      (Sect. 2.1, Eq. massmom)
  m2m_add  Q_a += sum_{b<=a} Qc_b g^(a-b)/(a-b)!  (Appendix A.1, Eq. massmomtrans)
  m2l_add  local += M2L(r = s_src - s_tgt, Q)     (Sect. 2.2, Eq. dmkdeffmm; M_k)
  l2l      local re-centred by h                  (Appendix A.2, Eq. gravmtranslat)
  l2p      field and potential polynomials at a  (Sect. 2.2)

Notation: multi-indices a = (ax, ay, az) in graded order (degree, then ax
descending, then ay descending); Q~_a = sum m b^a / a!; D_a = d^a (1/|r|).
The local expansion of a node holds
  H_g = (-1)^(|g|+1) sum_{|a| <= P+1-|g|} D_(a+g) Q~_a   for 1 <= |g| <= P+1
  P_b = (-1)^|b|     sum_{|a| <= P-|b|}   D_(a+b) Q~_a   for |b| <= P
stored as local[0 .. NH-2] = H (slots 1..NH-1) followed by local[NH-1 ..] = P.
The field at offset a from the centre is F_c = sum_b H_(b+e_c) a^b/b! and the
potential sum_b P_b a^b/b!; the caller multiplies both by -G.

D_a comes from the Laplace-kernel recurrence written for D itself:
  n |r|^2 D_a = -(2n-1) sum_c a_c r_c D_(a-e_c) - (n-1) sum_c a_c (a_c-1) D_(a-2e_c).
For |g| <= P the potential sum of P_g is a prefix of the field sum of H_g, so
both come out of one pass over a.
"""
import math
import os
import sys

PMAX = 4


def multi(n_max):
    out = []
    for n in range(n_max + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                out.append((a, b, n - a - b))
    return out


def ncoef(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def fac(a):
    return math.factorial(a[0]) * math.factorial(a[1]) * math.factorial(a[2])


def add(a, b):
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


def sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def lit(v):
    r = repr(float(v))
    return r


class Counter:
    def __init__(self):
        self.fma = 0
        self.mul = 0
        self.add = 0

    def flops(self):
        return 2 * self.fma + self.mul + self.add


def monomial_code(name, vec, deg, idx, lines, cnt, over_fact=True):
    """name[k] = vec^a / a! (or vec^a) for |a| <= deg, in graded order."""
    ms = multi(deg)
    lines.append(f"    double {name}[{len(ms)}];")
    lines.append(f"    {name}[0] = 1.0;")
    for k, a in enumerate(ms[1:], start=1):
        # build from the predecessor with the first positive component lowered
        c = 0 if a[0] > 0 else (1 if a[1] > 0 else 2)
        prev = list(a); prev[c] -= 1
        pk = idx[tuple(prev)]
        if over_fact and a[c] > 1:
            lines.append(f"    {name}[{k}] = {name}[{pk}] * ({vec}[{c}] * {lit(1.0 / a[c])});")
            cnt.mul += 2
        else:
            lines.append(f"    {name}[{k}] = {name}[{pk}] * {vec}[{c}];")
            cnt.mul += 1


def gen(P):
    NQ = ncoef(P)
    NH = ncoef(P + 1)
    NL = (NH - 1) + NQ
    ms = multi(P + 1)
    idx = {a: k for k, a in enumerate(ms)}
    out = []
    out.append(f"template <> struct Exp<{P}> {{")
    out.append(f"  static constexpr int P = {P};")
    out.append(f"  static constexpr int NQ = {NQ};   // mass moments, |a| <= P")
    out.append(f"  static constexpr int NL = {NL};   // local coefficients: H then P")

    # ---- P2M
    c = Counter()
    L = []
    L.append("  __device__ __forceinline__ static void p2m_add(const double* b, double m, double* Q) {")
    monomial_code("mb", "b", P, idx, L, c)
    for k in range(NQ):
        L.append(f"    Q[{k}] = fma(m, mb[{k}], Q[{k}]);")
        c.fma += 1
    L.append("  }")
    out += L
    out.append(f"  static constexpr int FLOPS_P2M = {c.flops()};")

    # ---- M2M
    c = Counter()
    L = ["  __device__ __forceinline__ static void m2m_add(const double* g, const double* Qc, double* Q) {"]
    monomial_code("mg", "g", P, idx, L, c)
    mq = multi(P)
    for k, a in enumerate(mq):
        terms = []
        for kb, b in enumerate(mq):
            d = sub(a, b)
            if min(d) < 0:
                continue
            terms.append((kb, idx[d]))
        expr = f"Q[{k}]"
        for kb, kd in terms:
            if kd == 0:
                expr = f"({expr} + Qc[{kb}])"
                c.add += 1
            else:
                expr = f"fma(Qc[{kb}], mg[{kd}], {expr})"
                c.fma += 1
        L.append(f"    Q[{k}] = {expr};")
    L.append("  }")
    out += L
    out.append(f"  static constexpr int FLOPS_M2M = {c.flops()};")

    # ---- M2L
    c = Counter()
    L = ["  __device__ __forceinline__ static void m2l_add(const double* r, const double* Q, double* local) {"]
    L.append("    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];")
    c.mul += 3; c.add += 2
    L.append("    const double rinv = rsqrt(r2);")
    L.append("    const double rinv2 = rinv * rinv;")
    c.mul += 1
    L.append(f"    double D[{NH}];")
    L.append("    D[0] = rinv;")
    for n in range(1, P + 2):
        L.append(f"    const double sn{n} = rinv2 * {lit(-1.0 / n)};")
        c.mul += 1
    for k, a in enumerate(ms[1:], start=1):
        n = sum(a)
        terms = []
        for cc in range(3):
            if a[cc] >= 1:
                b = list(a); b[cc] -= 1
                coef = (2 * n - 1) * a[cc]
                terms.append(f"{lit(coef)} * r[{cc}] * D[{idx[tuple(b)]}]")
                c.mul += 2
            if a[cc] >= 2:
                b = list(a); b[cc] -= 2
                coef = (n - 1) * a[cc] * (a[cc] - 1)
                terms.append(f"{lit(coef)} * D[{idx[tuple(b)]}]")
                c.mul += 1
        c.add += len(terms) - 1
        c.mul += 1
        L.append(f"    D[{k}] = ({' + '.join(terms)}) * sn{n};")
    # contractions
    for kg, g in enumerate(ms[1:], start=1):
        ng = sum(g)
        hslot = kg - 1
        # sum over a in graded order with |a| <= P+1-ng (a within mass-moment range)
        alist = [a for a in multi(P + 1 - ng)]
        acc = None
        lines_g = []
        first = True
        pdone = False
        for a in alist:
            na = sum(a)
            if ng <= P and not pdone and na > P - ng:
                # potential prefix complete
                lines_g.append(f"      local[{NH - 1 + kg}] {'+' if ng % 2 == 0 else '-'}= s;")
                c.add += 1
                pdone = True
            term_d = idx[add(a, g)]
            term_q = idx[a]
            if first:
                lines_g.append(f"      double s = D[{term_d}] * Q[{term_q}];")
                c.mul += 1
                first = False
            else:
                lines_g.append(f"      s = fma(D[{term_d}], Q[{term_q}], s);")
                c.fma += 1
        if ng <= P and not pdone:
            lines_g.append(f"      local[{NH - 1 + kg}] {'+' if ng % 2 == 0 else '-'}= s;")
            c.add += 1
        sign_h = '+' if (ng + 1) % 2 == 0 else '-'
        lines_g.append(f"      local[{hslot}] {sign_h}= s;")
        c.add += 1
        L.append("    {")
        L += lines_g
        L.append("    }")
    # P_0
    L.append("    {")
    first = True
    for a in multi(P):
        if first:
            L.append(f"      double s = D[{idx[a]}] * Q[{idx[a]}];")
            c.mul += 1
            first = False
        else:
            L.append(f"      s = fma(D[{idx[a]}], Q[{idx[a]}], s);")
            c.fma += 1
    L.append(f"      local[{NH - 1}] += s;")
    c.add += 1
    L.append("    }")
    L.append("  }")
    out += L
    out.append(f"  static constexpr int FLOPS_M2L = {c.flops()};  // + one rsqrt")
    # same contraction in FP32 (r and Q rounded to FP32), each term added to
    # the FP64 local expansion
    Lm = []
    for line in L:
        line = line.replace("static void m2l_add(const double* r, const double* Q, double* local)",
                            "static void m2l_add_f32(const float* r, const float* Q, double* local)")
        line = line.replace("const double ", "const float ").replace("double D[", "float D[")
        line = line.replace("double s = ", "float s = ")
        line = line.replace("rsqrt(r2)", "__frsqrt_rn(r2)")
        line = line.replace("fma(", "fmaf(")
        import re as _re
        line = _re.sub(r"(-?\d+\.\d+(e-?\d+)?)", r"\1f", line) if ("D[" in line and "=" in line and "local" not in line) or "sn" in line else line
        line = line.replace("local[", "local[").replace("] += s;", "] += (double)s;").replace("] -= s;", "] -= (double)s;")
        Lm.append(line)
    out += Lm

    # ---- M2L of one node pair in both directions (the one-sided symmetric
    # form): D(r) once for r = s_S - s_T; the target side as m2l_add; the
    # source side with D(-r) = (-1)^|k| D(r): with QTs the target's moments
    # with odd degrees negated (the caller's), H_g -= s and P_b += s, added to
    # outS atomically
    c = Counter()
    L = ["  __device__ __forceinline__ static void m2l_pair(const double* r, const double* QS,",
         "                                                    const double* QTs, double* local,",
         "                                                    double* outS) {"]
    body = []
    capture = False
    for line in out[out.index("  __device__ __forceinline__ static void m2l_add(const double* r, const double* Q, double* local) {") + 1:]:
        if line.startswith("    {") and not capture:
            capture = True
        if capture:
            break
        body.append(line)
    L += body  # r2, rinv, D recurrence
    # flops of the derivative part, from the same counts as m2l_add
    c.mul += 4; c.add += 2
    for k, a in enumerate(ms[1:], start=1):
        n = sum(a)
        nt = sum(1 for cc in range(3) if a[cc] >= 1) + sum(1 for cc in range(3) if a[cc] >= 2)
        c.mul += 2 * sum(1 for cc in range(3) if a[cc] >= 1) + sum(1 for cc in range(3) if a[cc] >= 2) + 1
        c.add += nt - 1
    c.mul += P + 1
    for side in ("T", "S"):
        Q = "QS" if side == "T" else "QTs"
        for kg, g in enumerate(ms[1:], start=1):
            ng = sum(g)
            hslot = kg - 1
            alist = [a for a in multi(P + 1 - ng)]
            lines_g = []
            first = True
            pdone = False
            def put(slot, sign):
                if side == "T":
                    return f"      local[{slot}] {sign}= s;"
                return f"      unsafeAtomicAdd(&outS[{slot}], {'-' if sign == '-' else ''}s);"
            for a in alist:
                na = sum(a)
                if ng <= P and not pdone and na > P - ng:
                    lines_g.append(put(NH - 1 + kg, ('+' if ng % 2 == 0 else '-') if side == "T" else '+'))
                    c.add += 1
                    pdone = True
                if first:
                    lines_g.append(f"      double s = D[{idx[add(a, g)]}] * {Q}[{idx[a]}];")
                    c.mul += 1
                    first = False
                else:
                    lines_g.append(f"      s = fma(D[{idx[add(a, g)]}], {Q}[{idx[a]}], s);")
                    c.fma += 1
            if ng <= P and not pdone:
                lines_g.append(put(NH - 1 + kg, ('+' if ng % 2 == 0 else '-') if side == "T" else '+'))
                c.add += 1
            lines_g.append(put(hslot, ('+' if (ng + 1) % 2 == 0 else '-') if side == "T" else '-'))
            c.add += 1
            L.append("    {")
            L += lines_g
            L.append("    }")
        L.append("    {")
        first = True
        for a in multi(P):
            if first:
                L.append(f"      double s = D[{idx[a]}] * {Q}[{idx[a]}];")
                c.mul += 1
                first = False
            else:
                L.append(f"      s = fma(D[{idx[a]}], {Q}[{idx[a]}], s);")
                c.fma += 1
        L.append(f"      local[{NH - 1}] += s;" if side == "T" else f"      unsafeAtomicAdd(&outS[{NH - 1}], s);")
        c.add += 1
        L.append("    }")
    L.append("  }")
    out += L
    out.append(f"  static constexpr int FLOPS_M2L_PAIR = {c.flops()};  // both directions, + one rsqrt")

    # ---- L2L (in place)
    c = Counter()
    L = ["  __device__ __forceinline__ static void l2l(const double* h, double* local) {"]
    monomial_code("mh", "h", P, idx, L, c)
    for kg, g in enumerate(ms[1:], start=1):
        ng = sum(g)
        expr = f"local[{kg - 1}]"
        for kd, d in enumerate(multi(P + 1 - ng)):
            if kd == 0:
                continue
            e = add(g, d)
            expr = f"fma(local[{idx[e] - 1}], mh[{kd}], {expr})"
            c.fma += 1
        L.append(f"    local[{kg - 1}] = {expr};")
    for kb, b in enumerate(multi(P)):
        nb = sum(b)
        expr = f"local[{NH - 1 + kb}]"
        for kd, d in enumerate(multi(P - nb)):
            if kd == 0:
                continue
            e = add(b, d)
            expr = f"fma(local[{NH - 1 + idx[e]}], mh[{kd}], {expr})"
            c.fma += 1
        L.append(f"    local[{NH - 1 + kb}] = {expr};")
    L.append("  }")
    out += L
    out.append(f"  static constexpr int FLOPS_L2L = {c.flops()};")

    # ---- L2P
    c = Counter()
    L = ["  __device__ __forceinline__ static void l2p(const double* a, const double* local, double* f, double& phi) {"]
    monomial_code("ma", "a", P, idx, L, c)
    for cc in range(3):
        e = [0, 0, 0]; e[cc] = 1
        expr = None
        for kb, b in enumerate(multi(P)):
            hk = idx[add(b, tuple(e))] - 1
            if expr is None:
                expr = f"local[{hk}]"
            else:
                expr = f"fma(local[{hk}], ma[{kb}], {expr})"
                c.fma += 1
        L.append(f"    f[{cc}] += {expr};")
        c.add += 1
    expr = None
    for kb, b in enumerate(multi(P)):
        if expr is None:
            expr = f"local[{NH - 1}]"
        else:
            expr = f"fma(local[{NH - 1 + kb}], ma[{kb}], {expr})"
            c.fma += 1
    L.append(f"    phi += {expr};")
    c.add += 1
    L.append("  }")
    out += L
    out.append(f"  static constexpr int FLOPS_L2P = {c.flops()};")
    out.append("};")
    return "\n".join(out)


def main(path):
    parts = [
        "// Generated by gen_expansions.py -- do not edit.",
        "// Cartesian expansion kernels for orders 0..%d (see the generator's docstring)." % PMAX,
        "#pragma once",
        "namespace sfmm {",
        "template <int P> struct Exp;",
    ]
    for P in range(PMAX + 1):
        parts.append(gen(P))
    parts.append("}  // namespace sfmm")
    text = "\n".join(parts) + "\n"
    old = open(path).read() if os.path.exists(path) else None
    if old != text:
        with open(path, "w") as f:
            f.write(text)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else
         os.path.join(os.path.dirname(os.path.abspath(__file__)), "expansions_gen.h"))
