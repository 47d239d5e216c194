"""Floating-point operation counts of the oracle's arithmetic (test and measurement infrastructure).

This is how the "algorithmic" FP64 work of the residual is defined: the operations of the plain
oracle, counted by running its own functions on a counting scalar, per unit of work the method
requires.  It is not part of the HIP path; only tests and the benchmark's documentation use it.

The counting scalar ``Op`` records each +, -, *, /, sqrt, log, log1p, exp (and powers) applied to it
as a node of an expression graph.  ``count`` walks the graph back from the outputs and counts each
reachable operation once, so

* a value computed but not used (the branch of a vectorised ``np.where`` that is not taken, e.g.
  the series or the direct form of the logarithmic mean) costs nothing;
* a subexpression the oracle computes once and reuses is counted once;
* a product with a literal 0 or +-1, or a sum with a literal 0, is not an operation (the structural
  zeros and ones of the viscous blocks C_mj, of the SBP operator, of the metric terms of an affine
  element are constants of the code, not data).
Negation and absolute value are sign operations and are not counted; comparisons decide branches
on the value and are not counted.

Units (per element of N^3 nodes, N = p + 1):
* ``pair``: one unordered node pair on a line, F#(q_i, q_j) contracted with A_l,i + A_l,j and added,
  weighted by D(i, j) and D(j, i), to both nodes (eq. discEL; the flux is symmetric, so the method
  evaluates it once per pair: 3 N^2 lines x N (N - 1) / 2 pairs per element);
* ``rest``: everything else of the residual of the oracle (interface SATs and dissipation, the
  viscous operator, the j = i volume terms, the combination and the division by J), per element.
The state used is uniform up to relative perturbations of 1e-4, so every logarithmic mean takes its
series form, as on the smooth workloads of the benchmark.
"""
from __future__ import annotations

import collections
import json
import math
import sys

import numpy as np

_COUNTED = ("add", "mul", "div", "sqrt", "log", "exp", "pow")


def _val(o):
    return o.v if isinstance(o, Op) else o


def _is_lit(o):
    return not isinstance(o, Op)


class Op:
    """A real number that remembers the operation that produced it (kind) and its operands."""

    __slots__ = ("v", "k", "a")

    def __init__(self, v, k=None, a=()):
        self.v = float(v)
        self.k = k
        self.a = a

    # -- arithmetic ------------------------------------------------------------------------
    def __add__(self, o):
        if _is_lit(o) and o == 0:
            return self
        return Op(self.v + _val(o), "add", (self, o) if isinstance(o, Op) else (self,))

    def __radd__(self, o):
        return self.__add__(o)

    def __sub__(self, o):
        if _is_lit(o) and o == 0:
            return self
        return Op(self.v - _val(o), "add", (self, o) if isinstance(o, Op) else (self,))

    def __rsub__(self, o):
        if _is_lit(o) and o == 0:
            return -self
        return Op(_val(o) - self.v, "add", (self,))

    def __mul__(self, o):
        if _is_lit(o):
            if o == 0:
                return 0.0
            if o == 1:
                return self
            if o == -1:
                return -self
        return Op(self.v * _val(o), "mul", (self, o) if isinstance(o, Op) else (self,))

    def __rmul__(self, o):
        return self.__mul__(o)

    def __truediv__(self, o):
        if _is_lit(o) and o == 1:
            return self
        return Op(self.v / _val(o), "div", (self, o) if isinstance(o, Op) else (self,))

    def __rtruediv__(self, o):
        if _is_lit(o) and o == 0:
            return 0.0
        return Op(_val(o) / self.v, "div", (self,))

    def __pow__(self, e):
        if e == 2:
            return Op(self.v * self.v, "mul", (self,))
        if e == 0.5:
            return self.sqrt()
        return Op(self.v ** e, "pow", (self,))

    def __neg__(self):
        return Op(-self.v, None, (self,))

    def __pos__(self):
        return self

    def __abs__(self):
        return Op(abs(self.v), None, (self,))

    # -- functions numpy calls on object arrays -------------------------------------------------
    def sqrt(self):
        return Op(math.sqrt(self.v), "sqrt", (self,))

    def log(self):
        return Op(math.log(self.v), "log", (self,))

    def log1p(self):
        return Op(math.log1p(self.v), "log", (self,))

    def exp(self):
        return Op(math.exp(self.v), "exp", (self,))

    def conjugate(self):
        return self

    @property
    def real(self):
        return self

    @property
    def imag(self):
        return 0.0

    # -- comparisons decide on the value --------------------------------------------------------
    def __lt__(self, o):
        return self.v < _val(o)

    def __le__(self, o):
        return self.v <= _val(o)

    def __gt__(self, o):
        return self.v > _val(o)

    def __ge__(self, o):
        return self.v >= _val(o)

    def __float__(self):
        return self.v


def _elementwise(name, fn):
    def f(x, *args, **kw):
        if isinstance(x, np.ndarray) and x.dtype == object:
            out = np.empty(x.shape, dtype=object)
            for idx, v in np.ndenumerate(x):
                out[idx] = getattr(v, name)() if isinstance(v, Op) else fn(float(v))
            return out
        if isinstance(x, Op):
            return getattr(x, name)()
        return getattr(np, name)(x, *args, **kw)
    return f


class _NumpyForCounting:
    """numpy with sqrt, log, log1p and exp that also take object arrays holding plain numbers next
    to counting scalars (a constant selected by np.where, a structural zero)."""

    sqrt = staticmethod(_elementwise("sqrt", math.sqrt))
    log = staticmethod(_elementwise("log", math.log))
    log1p = staticmethod(_elementwise("log1p", math.log1p))
    exp = staticmethod(_elementwise("exp", math.exp))

    def __getattr__(self, name):
        return getattr(np, name)


class counting_numpy:
    """Context in which the oracle modules use _NumpyForCounting (their code is unchanged)."""

    def __enter__(self):
        from . import gas, geometry, operators, residual
        self.mods = (gas, geometry, operators, residual)
        self.saved = [m.np for m in self.mods]
        for m in self.mods:
            m.np = _NumpyForCounting()
        return self

    def __exit__(self, *exc):
        for m, saved in zip(self.mods, self.saved):
            m.np = saved
        return False


def wrap(x):
    """An object array of counting scalars with the values of x (inputs: no operation)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape, dtype=object)
    flat = out.reshape(-1)
    for i, v in enumerate(x.reshape(-1)):
        flat[i] = Op(v)
    return out


def count(*outputs):
    """Operations reachable from the outputs (arrays or scalars), by kind; 'flop' is their sum."""
    seen = set()
    kinds = collections.Counter()
    stack = []
    for o in outputs:
        arr = np.asarray(o, dtype=object).reshape(-1)
        stack.extend(v for v in arr if isinstance(v, Op))
    while stack:
        n = stack.pop()
        if id(n) in seen:
            continue
        seen.add(id(n))
        if n.k is not None:
            kinds[n.k] += 1
        stack.extend(a for a in n.a if isinstance(a, Op))
    kinds["flop"] = sum(kinds[k] for k in _COUNTED)
    return kinds


def _smooth_state(N, K, gamma, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (K, N, N, N)
    rho = 1.0 + 1e-4 * rng.uniform(-1, 1, shape)
    u = 0.3 + 1e-4 * rng.uniform(-1, 1, (3,) + shape)
    P = 1.0 + 1e-4 * rng.uniform(-1, 1, shape)
    return np.stack([rho, rho * u[0], rho * u[1], rho * u[2], P / (gamma - 1.0) + 0.5 * rho * (u * u).sum(0)])


def unit_counts(p, viscous=True, gamma=1.4, R=1.0, mu=1e-3, Pr=0.72, eta=1.0, iface_diss=1):
    """Operation counts of the oracle per unit: one volume pair and the rest per element.

    Evaluated on one periodic element (its own neighbour across every face) with a warped mapping,
    so that no metric term is a literal constant."""
    from . import geometry, operators, residual as RS
    from . import gas as G
    N = p + 1
    sbp = operators.SBP1D(p)
    xi = sbp.x
    g = np.stack(np.meshgrid(xi, xi, xi, indexing="ij"))          # (3, N, N, N) as (i1, i2, i3)
    g = np.transpose(g, (0, 3, 2, 1))                               # axes (i3, i2, i1)
    x = g + 0.05 * np.sin(np.pi * g[[1, 2, 0]]) * np.cos(np.pi * g[[2, 0, 1]])
    x = x[:, None]                                                  # one element
    metric = geometry.curl_metrics(x, sbp.D)
    jac = geometry.jacobian(x, sbp.D)
    nbr = np.zeros((1, 6), dtype=np.int64)
    prm = RS.Params(gamma, R, mu if viscous else 0.0, Pr, eta, iface_diss, 0)
    q = wrap(_smooth_state(N, 1, gamma))
    m_o, j_o = wrap(metric), wrap(jac)
    with counting_numpy():
        total = count(RS.residual(q, m_o, j_o, nbr, sbp, prm))
        vol = count(RS.volume_term(q, m_o, sbp, prm))
        # one unordered pair: the contracted flux and its two weighted contributions
        qa, qb = q[:, 0, 0, 0, 0], q[:, 0, 0, 0, 1]
        n = m_o[0:3, 0, 0, 0, 0] + m_o[0:3, 0, 0, 0, 1]
        f = G.contract(G.TWO_POINT[0](qa[:, None], qb[:, None], prm.gas), n[:, None])[:, 0]
        pair = count(*[sbp.D[0, 1] * fc for fc in f], *[sbp.D[1, 0] * fc for fc in f])
    pair["add"] += 10                     # the two accumulations into the nodes' sums
    pair["flop"] += 10
    rest = collections.Counter({k: total[k] - vol[k] for k in set(total) | set(vol)})
    pairs_per_elem = 3 * N * N * N * (N - 1) // 2
    return {"p": p, "viscous": viscous, "pair": dict(pair), "rest_per_element": dict(rest),
            "pairs_per_element": pairs_per_elem,
            "flop_per_element": pairs_per_elem * pair["flop"] + rest["flop"],
            "flop_per_node": (pairs_per_elem * pair["flop"] + rest["flop"]) / N ** 3,
            "oracle_volume_flop_per_element": vol["flop"]}


if __name__ == "__main__":
    degrees = [int(v) for v in sys.argv[1:]] or [4]
    out = [unit_counts(p, viscous=v) for p in degrees for v in (True, False)]
    print(json.dumps(out, indent=1))
