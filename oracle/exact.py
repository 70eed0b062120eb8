"""Exact-rational brute-force renderer for tiny inputs (test infrastructure only).

Every input number (voxel, table entry, rotation entry, extent, window, step,
tau) is converted exactly from its binary floating-point value into a
``fractions.Fraction``; every step of the ray-casting definition (paper
Sec. 2 and Sec. 2.4, with the readings stated in ``vr_oracle.c``) is then
evaluated without rounding, sample by sample:

* pixel centre -> orthographic ray (rows of R are the view axes), or the
  perspective ray from the eye at c - D e3 through the pixel's point on the
  plane through c (its unit direction needs a square root: it is taken to 60
  significant digits and then used as an exact rational, so the result is the
  exact image of a direction within 1e-55 of the true one);
* ray/box interval by solving 0 <= o_i + t d_i <= n_i - 1 per axis;
* lattice t_k = t_in + (k + 1/2) step while t_k < t_out;
* owner sub-volume by searching the ownership boxes;
* trilinear value as an explicit 8-corner weighted sum;
* transfer-function lookup (opacity times the channel mask interpolated
  along axis 3, when one is given), front-to-back emission-absorption, ERT test;
* per-ray ordering of the partial results by their first sample, then the
  over operator (paper Sec. 2.5).

Derivatives: ``Dual`` numbers carry one directional derivative through the
same evaluation (forward mode), independent of the reverse-mode recursion the
FP64 oracle and the GPU adjoint use.

Only for volumes of a few hundred voxels and images of a few dozen pixels.
"""
from __future__ import annotations

from decimal import Decimal, localcontext
from fractions import Fraction as Fr
import math


class Dual:
    """Value + one directional derivative, both exact rationals."""
    __slots__ = ("v", "d")

    def __init__(self, v, d=Fr(0)):
        self.v = v if isinstance(v, Fr) else Fr(v)
        self.d = d if isinstance(d, Fr) else Fr(d)

    def __add__(self, o):
        o = o if isinstance(o, Dual) else Dual(o)
        return Dual(self.v + o.v, self.d + o.d)

    __radd__ = __add__

    def __sub__(self, o):
        o = o if isinstance(o, Dual) else Dual(o)
        return Dual(self.v - o.v, self.d - o.d)

    def __rsub__(self, o):
        return Dual(o) - self

    def __mul__(self, o):
        o = o if isinstance(o, Dual) else Dual(o)
        return Dual(self.v * o.v, self.v * o.d + self.d * o.v)

    __rmul__ = __mul__

    def scale(self, k: Fr):
        return Dual(self.v * k, self.d * k)


def _fr(x) -> Fr:
    return Fr(float(x))


def _ray_interval(o, d, n):
    """Exact [t_in, t_out] of the ray inside [0, n_i - 1]^3, or None on a miss."""
    tin, tout = None, None
    for i in range(3):
        lo, hi = Fr(0), Fr(n[i] - 1)
        if d[i] == 0:
            if o[i] < lo or o[i] > hi:
                return None
            continue
        a, b = (lo - o[i]) / d[i], (hi - o[i]) / d[i]
        a, b = min(a, b), max(a, b)
        tin = a if tin is None else max(tin, a)
        tout = b if tout is None else min(tout, b)
    if tin is None or not tin < tout:
        return None
    return tin, tout


def _owner(p, boxes):
    for j, (lo, hi, cl) in enumerate(boxes):
        ok = True
        for i in range(3):
            if p[i] < lo[i]:
                ok = False
            elif (p[i] > hi[i]) if cl[i] else (p[i] >= hi[i]):
                ok = False
        if ok:
            return j
    return None


def _sqrt(q: Fr) -> Fr:
    with localcontext() as ctx:
        ctx.prec = 60
        return Fr((Decimal(q.numerator) / Decimal(q.denominator)).sqrt())


def render(vol, tf, R, W, H, extent, vmin, vmax, step=0.5, tau=0.99, boxes=None,
           dvol=None, dtf=None, mip=False, eye_dist=0.0, mask=None):
    """Exact image [H][W][4] as Fractions (or Duals when dvol/dtf give a direction).

    mip=True: maximum intensity projection (M, M, M, M), M = max over samples of
    the normalised value clamped to [0, 1] (Fractions only).

    vol: nested [n3][n2][n1] numbers; tf: [M][4]; R: 3x3; boxes: optional list of
    (lo, hi, closed) ownership boxes.  Returns a list of rows of pixel tuples.
    """
    n3, n2, n1 = len(vol), len(vol[0]), len(vol[0][0])
    n = (n1, n2, n3)
    use_dual = dvol is not None or dtf is not None
    V = [[[None] * n1 for _ in range(n2)] for _ in range(n3)]
    for z in range(n3):
        for y in range(n2):
            for x in range(n1):
                v = _fr(vol[z][y][x])
                if use_dual:
                    V[z][y][x] = Dual(v, _fr(dvol[z][y][x]) if dvol is not None else 0)
                else:
                    V[z][y][x] = v
    M = len(tf)
    T_ = []
    for i in range(M):
        row = []
        for c in range(4):
            v = _fr(tf[i][c])
            row.append(Dual(v, _fr(dtf[i][c]) if dtf is not None else 0) if use_dual else v)
        T_.append(row)
    Rf = [[_fr(R[r][c]) for c in range(3)] for r in range(3)]
    e1, e2, e3 = Rf[0], Rf[1], Rf[2]
    S = _fr(extent)
    D = _fr(eye_dist)
    lo_w, hi_w = _fr(vmin), _fr(vmax)
    dt, tau_f = _fr(step), _fr(tau)
    ert = tau_f < 1
    cen = [Fr(n[i] - 1, 2) for i in range(3)]
    bx = None
    if boxes is not None:
        bx = [(tuple(Fr(a) for a in lo), tuple(Fr(a) for a in hi), tuple(cl)) for lo, hi, cl in boxes]

    def value_at(p):
        base, frac = [], []
        for i in range(3):
            k = math.floor(p[i])
            k = max(0, min(n[i] - 2, k))
            base.append(k)
            frac.append(p[i] - k)
        acc = None
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    w = ((frac[0] if dx else 1 - frac[0]) * (frac[1] if dy else 1 - frac[1])
                         * (frac[2] if dz else 1 - frac[2]))
                    term = V[base[2] + dz][base[1] + dy][base[0] + dx]
                    term = term.scale(w) if use_dual else term * w
                    acc = term if acc is None else acc + term
        return acc

    mk = None if mask is None else [_fr(x) for x in mask]

    def mask_at(p):
        """Channel weight: the mask interpolated along axis 3 with the trilinear weight."""
        if mk is None:
            return Fr(1)
        k = max(0, min(n[2] - 2, math.floor(p[2])))
        f = p[2] - k
        return (1 - f) * mk[k] + f * mk[k + 1]

    def classify(val):
        vv = val.v if use_dual else val
        if hi_w > lo_w:
            s_raw = (vv - lo_w) / (hi_w - lo_w)
        else:
            s_raw = Fr(0)
        if s_raw <= 0:
            s = Fr(0)
            s_d = Dual(Fr(0)) if use_dual else Fr(0)
        elif s_raw >= 1:
            s = Fr(1)
            s_d = Dual(Fr(1)) if use_dual else Fr(1)
        else:
            s = s_raw
            s_d = (val - lo_w).scale(1 / (hi_w - lo_w)) if use_dual else s_raw
        u = s * (M - 1)
        i = min(math.floor(u), M - 2)
        if use_dual:
            u_d = s_d.scale(Fr(M - 1))
            w = u_d - Fr(i)
            return [T_[i][c] * (1 - w) + T_[i + 1][c] * w for c in range(4)]
        w = u - i
        return [(1 - w) * T_[i][c] + w * T_[i + 1][c] for c in range(4)]

    zero = Dual(Fr(0)) if use_dual else Fr(0)
    one = Dual(Fr(1)) if use_dual else Fr(1)
    image = []
    for v in range(H):
        row = []
        for u in range(W):
            x = (Fr(2 * u + 1, 2 * W) - Fr(1, 2)) * S
            y = (Fr(2 * v + 1, 2 * H) - Fr(1, 2)) * S * Fr(H, W)
            if D > 0:
                o = [cen[i] - D * e3[i] for i in range(3)]
                w = [x * e1[i] + y * e2[i] + D * e3[i] for i in range(3)]
                ln = _sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2])
                d = [w[i] / ln for i in range(3)]
            else:
                o = [cen[i] + x * e1[i] + y * e2[i] - S * e3[i] for i in range(3)]
                d = e3
            iv = _ray_interval(o, d, n)
            if iv is None:
                row.append((zero, zero, zero, zero))
                continue
            tin, tout = iv
            if mip:
                m = Fr(0)
                k = 0
                while True:
                    t = tin + (k + Fr(1, 2)) * dt
                    if not t < tout:
                        break
                    p = [o[i] + t * d[i] for i in range(3)]
                    if bx is not None and _owner(p, bx) is None:
                        raise AssertionError("sample inside the volume owned by no box")
                    s_raw = (value_at(p) - lo_w) / (hi_w - lo_w) if hi_w > lo_w else Fr(0)
                    m = max(m, min(Fr(1), max(Fr(0), s_raw)) * mask_at(p))
                    k += 1
                row.append((m, m, m, m))
                continue
            chains = {}  # owner -> [C(3), T, stopped, tfirst]
            k = 0
            while True:
                t = tin + (k + Fr(1, 2)) * dt
                if not t < tout:
                    break
                p = [o[i] + t * d[i] for i in range(3)]
                key = 0
                if bx is not None:
                    key = _owner(p, bx)
                    if key is None:
                        raise AssertionError("sample inside the volume owned by no box")
                ch = chains.get(key)
                if ch is None:
                    ch = [[zero, zero, zero], one, False, t]
                    chains[key] = ch
                if not ch[2]:
                    r, g, b, a = classify(value_at(p))
                    a = a * mask_at(p)
                    Tv = ch[1]
                    ch[0] = [ch[0][0] + Tv * a * r, ch[0][1] + Tv * a * g, ch[0][2] + Tv * a * b]
                    ch[1] = Tv * (1 - a)
                    Tval = ch[1].v if use_dual else ch[1]
                    if ert and 1 - Tval >= tau_f:
                        ch[2] = True
                k += 1
            order = sorted(chains.values(), key=lambda c: c[3])
            Cc = [zero, zero, zero]
            A = zero
            for ch in order:
                Ab = 1 - ch[1]
                Cc = [Cc[c] + (1 - A) * ch[0][c] for c in range(3)]
                A = A + (1 - A) * Ab
            row.append((Cc[0], Cc[1], Cc[2], A))
        image.append(row)
    return image


def to_float(image):
    """Fractions (or Duals) -> nested floats; Duals give (value, derivative) pairs."""
    out = []
    for row in image:
        r = []
        for px in row:
            if isinstance(px[0], Dual):
                r.append(tuple((float(c.v), float(c.d)) for c in px))
            else:
                r.append(tuple(float(c) for c in px))
        out.append(r)
    return out
