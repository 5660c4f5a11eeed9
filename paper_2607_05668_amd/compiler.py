"""Conservation law -> collide-and-stream scheme: a host-side compiler slice.

The paper derives its lattice Boltzmann schemes from a declared
conservation law (Sec. 2.5, Alg. 1): a Buckingham-Pi projection reads the
lattice scaling of every quantity off its SI dimension, *Split* sends the
terms under a divergence to the flux and the rest to the source, *Cascade*
replaces every spatial gradient in a flux or source by a gradient tracker
(Sec. 2.1.1: a linear advection-relaxation field whose equilibrium encodes
the gradient), expanding gradients of derived quantities over the conserved
states by the chain rule first, and *Assemble* gives every field of the
resulting gradient-free system its own populations with the exact-flux
equilibrium and a relaxation slot.  This module implements those passes on
SymPy expressions and emits the result as a device functor for the step
kernel of this library (flux, deviation of the flux from its reference
value, source), plus the numpy form the tests compare against the oracle.

Declaring a system::

    m = Model("euler2d", dim=2)
    rho = m.state("rho", DENSITY)
    mom = m.state("m", DENSITY * VELOCITY, rank=1)
    E = m.state("E", PRESSURE)
    gamma = m.param("gamma", ONE)
    u = mom / rho
    p = (gamma - 1) * (E - dot(mom, u) / 2)
    m.law(dt(rho) + div(mom))
    m.law(dt(mom) + div(outer(mom, u) + p * eye(2)))
    m.law(dt(E) + div((E + p) * u))
    scheme = m.compile()

``grad(V)`` may appear anywhere in a law; ``m.tracker_velocity(u)`` sets the
velocity the gradient trackers are advected with.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction

import sympy as sp
from sympy.printing.cxx import CXX17CodePrinter
from sympy.printing.precedence import PRECEDENCE

# --------------------------------------------------------------------------
# SI dimensions and the Buckingham-Pi projection onto the lattice scales
# --------------------------------------------------------------------------
BASE = ("L", "T", "M", "Theta")


@dataclass(frozen=True)
class Dim:
    """Exponents over the base dimensions (length, time, mass, temperature)."""
    e: tuple = (0, 0, 0, 0)

    def __mul__(self, o):
        return Dim(tuple(Fraction(a) + Fraction(b) for a, b in zip(self.e, o.e)))

    def __truediv__(self, o):
        return Dim(tuple(Fraction(a) - Fraction(b) for a, b in zip(self.e, o.e)))

    def __pow__(self, k):
        return Dim(tuple(Fraction(a) * Fraction(k) for a in self.e))


ONE = Dim()
LENGTH = Dim((1, 0, 0, 0))
TIME = Dim((0, 1, 0, 0))
MASS = Dim((0, 0, 1, 0))
TEMPERATURE = Dim((0, 0, 0, 1))
VELOCITY = LENGTH / TIME
DENSITY = MASS / LENGTH ** 3
PRESSURE = MASS / LENGTH / TIME ** 2
DYNAMIC_VISCOSITY = PRESSURE * TIME
THERMAL_CONDUCTIVITY = MASS * LENGTH / TIME ** 3 / TEMPERATURE
GAS_CONSTANT = LENGTH ** 2 / TIME ** 2 / TEMPERATURE


def pq_projection(references):
    """The map D(X) -> (p, q) of the Buckingham-Pi step: with B the matrix
    whose columns are the base exponents of length, time and each reference
    quantity (which must together span the base dimensions), (p, q) =
    [I_2 | 0] B^-1 D(X), so that X_phys = X_lattice dx^p dt^q."""
    cols = [LENGTH.e, TIME.e] + [r.e for r in references]
    B = sp.Matrix([[sp.Rational(Fraction(c[i]).numerator, Fraction(c[i]).denominator) for c in cols]
                   for i in range(len(BASE))])
    if B.shape[0] != B.shape[1] or B.det() == 0:
        raise ValueError("length, time and the references must form a basis of the base dimensions")
    Binv = B.inv()

    def pq(d: Dim):
        v = sp.Matrix([sp.Rational(Fraction(x).numerator, Fraction(x).denominator) for x in d.e])
        c = Binv * v
        return (c[0], c[1])
    return pq


# --------------------------------------------------------------------------
# Operators of the declaration language
# --------------------------------------------------------------------------
class Partial(sp.Function):
    """Unevaluated spatial derivative d V / d x_axis of a scalar expression."""
    nargs = 2


def grad(v):
    """Gradient of a scalar (column vector) or of a vector (rows d v_a / d x_b)."""
    if isinstance(v, sp.MatrixBase):
        return sp.Matrix(v.shape[0], _DIM[0], lambda a, b: Partial(v[a], b))
    return sp.Matrix(_DIM[0], 1, lambda b, _: Partial(v, b))


def outer(a, b):
    return a * b.T


def dot(a, b):
    return (a.T * b)[0, 0]


def eye(d):
    return sp.eye(d)


def trace(t):
    return t.trace()


_DIM = [2]          # dimension of the model being declared (grad needs it)


class Terms:
    """A law's terms: the time derivative of one state, terms under a
    divergence, and the remaining (source) terms, all on the left-hand side."""

    def __init__(self, dt=None, div=(), rest=None):
        self.dt, self.div, self.rest = dt, list(div), rest

    @staticmethod
    def _lift(o):
        return o if isinstance(o, Terms) else Terms(rest=o)

    def __add__(self, o):
        o = Terms._lift(o)
        if self.dt is not None and o.dt is not None:
            raise ValueError("a law has one time derivative")
        rest = o.rest if self.rest is None else (self.rest if o.rest is None else self.rest + o.rest)
        return Terms(self.dt if self.dt is not None else o.dt, self.div + o.div, rest)

    __radd__ = __add__

    def __neg__(self):
        if self.dt is not None:
            raise ValueError("the time derivative keeps a positive sign")
        return Terms(None, [-d for d in self.div], None if self.rest is None else -self.rest)

    def __sub__(self, o):
        return self + (-Terms._lift(o))

    def __rsub__(self, o):
        return Terms._lift(o) + (-self)


def dt(q):
    return Terms(dt=q)


def div(t):
    return Terms(div=[t])


# --------------------------------------------------------------------------
# Model declaration
# --------------------------------------------------------------------------
@dataclass
class Quantity:
    name: str
    dim: Dim
    symbols: list            # component symbols
    rank: int


@dataclass
class Scheme:
    """The compiled, gradient-free system over Q+ (conserved fields, then
    trackers): flux rows Phi[k] (D components each), sources S[k], all
    algebraic in the field symbols ``fields``, the parameters and 1/tau_grad."""
    name: str
    dim: int
    fields: list                     # field symbols, conserved then trackers
    names: list
    n_conserved: int
    flux: list                       # [K][D] sympy expressions
    source: list                     # [K]
    params: list                     # parameter symbols (kernel order)
    param_names: list
    inv_tau_grad: sp.Symbol
    pq: dict                         # field / parameter name -> (p, q)
    parents: dict = field(default_factory=dict)   # tracker name -> parent expression
    dims: dict = field(default_factory=dict)      # field / parameter name -> SI dimension (Dim)

    @property
    def K(self):
        return len(self.fields)

    def tracker(self, k):
        return k >= self.n_conserved

    def numpy_flux_source(self):
        """(flux(q, par, inv_tg) -> [K, D], source(q, par, inv_tg) -> [K])."""
        import numpy as np
        args = [list(self.fields), list(self.params), self.inv_tau_grad]
        fF = sp.lambdify(args, [list(r) for r in self.flux], "numpy")
        fS = sp.lambdify(args, list(self.source), "numpy")
        return (lambda q, par, itg: np.array(fF(list(q), list(par), itg), dtype=float),
                lambda q, par, itg: np.array(fS(list(q), list(par), itg), dtype=float))


class Model:
    def __init__(self, name: str, dim: int = 2):
        self.name, self.dim = name, dim
        _DIM[0] = dim
        self.states: list[Quantity] = []
        self.parameters: list[Quantity] = []
        self.laws: list[Terms] = []
        self.velocity = None
        self.tracked_exprs: dict = {}   # symbol -> derived expression tracked as an auxiliary field
        self.tracked_dims: dict = {}    # symbol -> its SI dimension, when declared
        self.tracked_vectors: dict = {} # name -> component symbols of a tracked vector
        self.tau_grad = sp.Symbol("tau_grad", positive=True)

    def state(self, name, dim: Dim, rank: int = 0):
        if rank == 0:
            syms = [sp.Symbol(name, real=True)]
            obj = syms[0]
        else:
            syms = [sp.Symbol(f"{name}{a}", real=True) for a in range(self.dim)]
            obj = sp.Matrix(syms)
        self.states.append(Quantity(name, dim, syms, rank))
        return obj

    def param(self, name, dim: Dim):
        s = sp.Symbol(name, real=True)
        self.parameters.append(Quantity(name, dim, [s], 0))
        return s

    def law(self, terms: Terms):
        if terms.dt is None:
            raise ValueError("a law needs the time derivative of a state")
        self.laws.append(terms)

    def tracker_velocity(self, u):
        self.velocity = u

    def tracked(self, name, expr, dim: Dim = None):
        """A derived quantity whose gradient is tracked directly (instead of
        expanded over the conserved states by the chain rule): returns the
        symbol(s) to use in the laws; they stand for ``expr`` everywhere.
        ``dim`` (its SI dimension) gives its trackers their lattice scaling."""
        if isinstance(expr, sp.MatrixBase):
            syms = [sp.Symbol(f"{name}{a}", real=True) for a in range(expr.shape[0])]
            for sy, e in zip(syms, expr):
                self.tracked_exprs[sy] = e
                if dim is not None:
                    self.tracked_dims[sy] = dim
            self.tracked_vectors[name] = syms
            return sp.Matrix(syms)
        sy = sp.Symbol(name, real=True)
        self.tracked_exprs[sy] = expr
        if dim is not None:
            self.tracked_dims[sy] = dim
        return sy

    # ---- passes ---------------------------------------------------------
    def _split(self):
        """Split: per state component, the flux (sum of the divergence terms)
        and the source (minus the remaining terms)."""
        D = self.dim
        out = {}
        for law in self.laws:
            q = law.dt
            comps = list(q) if isinstance(q, sp.MatrixBase) else [q]
            for a, s in enumerate(comps):
                F = [sp.Integer(0)] * D
                for t in law.div:
                    if isinstance(q, sp.MatrixBase):
                        row = t[a, :] if t.shape[1] == D else t.T[a, :]
                        F = [F[c] + row[c] for c in range(D)]
                    else:
                        F = [F[c] + t[c] for c in range(D)]
                S = sp.Integer(0)
                if law.rest is not None:
                    r = law.rest
                    S = -(r[a] if isinstance(r, sp.MatrixBase) else r)
                out[s] = (F, S)
        order = [s for q in self.states for s in q.symbols]
        missing = [s for s in order if s not in out]
        if missing:
            raise ValueError(f"no law for {missing}")
        return order, out

    def compile(self, references=(DENSITY, GAS_CONSTANT), strain=None):
        """Run Split, Cascade and Assemble.  references: the characteristic
        reference quantities of the Buckingham-Pi step; strain: the name of
        a tracked velocity whose gradient enters only through its symmetric
        part, to be carried by D(D+1)/2 strain trackers (Alg. 1's optional
        strain reduction)."""
        D = self.dim
        order, split = self._split()
        state_set = set(order)
        tracked_syms = dict(self.tracked_exprs)
        parents_order = list(order) + list(tracked_syms)
        trackers = {}                 # parent symbol -> list of D tracker symbols
        parent_expr = {}

        def tracker_for(V):
            if V not in trackers:
                trackers[V] = [sp.Symbol(f"G_{V}_{b}", real=True) for b in range(D)]
                parent_expr[V] = tracked_syms.get(V, V)
            return trackers[V]

        def resolve(expr):
            """Replace every Partial(V, b), innermost first (Cascade)."""
            while True:
                parts = sorted(expr.atoms(Partial), key=sp.count_ops)
                if not parts:
                    return expr
                P = parts[0]
                V, b = P.args
                b = int(b)
                if V.atoms(Partial):
                    expr = expr.subs(P, Partial(resolve(V), b))
                    continue
                tracker_syms = {g: par for par, gs in trackers.items() for g in gs}
                if V in state_set or V in tracked_syms or V in tracker_syms:
                    rep = tracker_for(V)[b]
                elif not (V.free_symbols & (state_set | set(tracked_syms) | set(tracker_syms))):
                    rep = sp.Integer(0)          # parameters only: constant in space
                else:
                    # derived: chain rule over the fields it is made of
                    rep = sum(sp.diff(V, x) * Partial(x, b) for x in V.free_symbols
                              if x in state_set or x in tracked_syms or x in tracker_syms)
                expr = expr.subs(P, rep)

        flux = {s: [resolve(sp.sympify(F)) for F in split[s][0]] for s in order}
        source = {s: resolve(sp.sympify(split[s][1])) for s in order}
        # gradient advection-relaxation laws of the trackers, until closed
        u = self.velocity
        itg = sp.Symbol("inv_tau_grad", positive=True)
        done = set()
        while len(done) < len(trackers):
            V = next(v for v in trackers if v not in done)
            done.add(V)
            if u is None:
                raise ValueError("declare the trackers' advection velocity (tracker_velocity)")
            for b, g in enumerate(trackers[V]):
                row = [g * u[c] - (parent_expr[V] * itg if b == c else 0) for c in range(D)]
                flux[g] = [resolve(sp.sympify(e)) for e in row]
                source[g] = -g * itg
        # field order: conserved states, then trackers by parent (states in
        # declaration order, tracked quantities, then trackers of trackers)
        rank = {v: i for i, v in enumerate(parents_order)}
        tracker_parents = sorted(trackers, key=lambda v: rank.get(v, len(rank) + list(trackers).index(v)))
        fields = list(order) + [g for v in tracker_parents for g in trackers[v]]
        names = {}
        if strain is not None:
            fields, flux, source, names = _strain_reduce(self, strain, trackers, fields, flux, source, itg, D)
        subs = dict(tracked_syms)
        subs[self.tau_grad] = 1 / itg
        F = [[sp.sympify(e).subs(subs) for e in flux[f]] for f in fields]
        S = [sp.sympify(source[f]).subs(subs) for f in fields]
        # lattice scaling of every field and parameter (Buckingham-Pi)
        pq_of = pq_projection(list(references))
        pq = {}
        for q in self.states:
            for sy in q.symbols:
                pq[str(sy)] = pq_of(q.dim)
        for q in self.parameters:
            pq[q.name] = pq_of(q.dim)
        dims = {}
        for q in self.states:
            for sy in q.symbols:
                dims[str(sy)] = q.dim
        for q in self.parameters:
            dims[q.name] = q.dim
        for v in tracker_parents:
            parent_dim = dims.get(str(v)) if v in state_set else self.tracked_dims.get(v)
            base = None if parent_dim is None else pq_of(parent_dim)
            for g in trackers[v]:
                pq[str(g)] = None if base is None else (base[0] - 1, base[1])
                if parent_dim is not None:
                    dims[str(g)] = parent_dim / LENGTH
        for f in fields:                   # strain trackers: the parent velocity's gradient
            if str(f) in names:
                pdim = self.tracked_dims.get(names[str(f)])
                pq[str(f)] = None if pdim is None else pq_of(pdim / LENGTH)
                if pdim is not None:
                    dims[str(f)] = pdim / LENGTH
        return Scheme(self.name, D, fields, [str(f) for f in fields], len(order), F, S,
                      [q.symbols[0] for q in self.parameters], [q.name for q in self.parameters], itg, pq,
                      {str(v): parent_expr[v] for v in tracker_parents}, dims)


def _strain_reduce(model, name, trackers, fields, flux, source, itg, D):
    """Alg. 1's optional strain reduction.  The velocity-gradient trackers
    G_ab (gradient of the tracked vector ``name``, d_b u_a) are replaced by
    the strain trackers S_ab = (G_ab + G_ba)/2, a <= b, provided every other
    flux and source depends on G only through its symmetric part: with
    G_ab = S_ab + W_ab, W antisymmetric, nothing may depend on W.  The
    trackers' own laws are linear in G with the common advection velocity,
    so the symmetrised laws close over S: flux (Phi_G_ab + Phi_G_ba)/2,
    source (S_G_ab + S_G_ba)/2.  Order (00, 11, 22, 01, 02, 12) in 3D,
    (00, 11, 01) in 2D.  Returns the new (fields, flux, source, strain name
    -> parent symbol)."""
    if name not in model.tracked_vectors:
        raise ValueError(f"strain reduction needs the tracked vector '{name}'")
    comps = model.tracked_vectors[name]
    G = [[trackers[comps[a]][b] if comps[a] in trackers else None for b in range(D)] for a in range(D)]
    if any(g is None for row in G for g in row):
        raise ValueError(f"the gradient of '{name}' is not tracked in full")
    pairs = [(a, a) for a in range(D)] + [(a, b) for a in range(D) for b in range(a + 1, D)]
    Ssym = {(a, b): sp.Symbol(f"S_{name}_{a}{b}", real=True) for a, b in pairs}
    W = {(a, b): sp.Symbol(f"W_{name}_{a}{b}", real=True) for a, b in pairs if a != b}
    rep = {}
    for a in range(D):
        for b in range(D):
            if a == b:
                rep[G[a][b]] = Ssym[(a, a)]
            elif a < b:
                rep[G[a][b]] = Ssym[(a, b)] + W[(a, b)]
            else:
                rep[G[a][b]] = Ssym[(b, a)] - W[(b, a)]
    gset = set(rep)

    def sym_only(e, what):
        r = sp.expand(sp.sympify(e).xreplace(rep))
        if r.free_symbols & set(W.values()):
            raise ValueError(f"{what} depends on the antisymmetric part of grad {name}: no strain reduction")
        return r
    nflux, nsource = {}, {}
    for f in fields:
        if f in gset:
            continue
        nflux[f] = [sym_only(e, f"the flux of {f}") for e in flux[f]]
        nsource[f] = sym_only(source[f], f"the source of {f}")
    names = {}
    for a, b in pairs:
        g1, g2 = G[a][b], G[b][a]
        sab = Ssym[(a, b)]
        nflux[sab] = [sym_only((flux[g1][c] + flux[g2][c]) / 2, f"the strain tracker {sab}") for c in range(D)]
        nsource[sab] = sym_only((sp.sympify(source[g1]) + source[g2]) / 2, f"the strain tracker {sab}")
        names[str(sab)] = comps[a]
    first = min(i for i, f in enumerate(fields) if f in gset)
    rest = [f for f in fields if f not in gset]
    nfields = rest[:first] + [Ssym[pr] for pr in pairs] + rest[first:]
    return nfields, nflux, nsource, names


# --------------------------------------------------------------------------
# Dedimensionalize: SI values -> nondimensional values -> lattice values
# --------------------------------------------------------------------------
def value_scale(d: Dim, characteristics):
    """The characteristic value of dimension d built from characteristic
    quantities [(Dim, SI value), ...] that span the base dimensions (e.g. a
    length, a sound speed, a density and a gas constant): with B the matrix
    of their exponent columns, d = B c and the scale is prod_j value_j^c_j."""
    cols = [c[0].e for c in characteristics]
    B = sp.Matrix([[sp.Rational(Fraction(c[i]).numerator, Fraction(c[i]).denominator) for c in cols]
                   for i in range(len(BASE))])
    if B.shape[0] != B.shape[1] or B.det() == 0:
        raise ValueError("the characteristic quantities must form a basis of the base dimensions")
    v = sp.Matrix([sp.Rational(Fraction(x).numerator, Fraction(x).denominator) for x in d.e])
    c = B.inv() * v
    out = 1.0
    for (dim, val), ex in zip(characteristics, c):
        out *= float(val) ** float(ex)
    return out


def nondimensional(scheme: Scheme, si_values: dict, characteristics):
    """Parameter values of the scheme in units of the characteristic scales
    (the value non-dimensionalization of the supplement's SI listing):
    X* = X_SI / value_scale(D(X))."""
    return {n: si_values[n] / value_scale(scheme.dims[n], characteristics) for n in si_values}


def lattice_values(scheme: Scheme, values: dict, dx: float, dt: float):
    """Alg. 1, Dedimensionalize: a quantity X with scaling (p, q) becomes
    X dx^-p dt^-q on the lattice (dx = dt = 1 there).  values: name ->
    value in the units the grid spacings dx, dt are measured in."""
    out = {}
    for n, v in values.items():
        p, q = scheme.pq[n]
        out[n] = float(v) * float(dx) ** (-float(p)) * float(dt) ** (-float(q))
    return out


def field_factors(scheme: Scheme, dx: float, dt: float):
    """Per-field factors dx^-p dt^-q taking the fields (conserved and
    trackers) to lattice units."""
    return [float(dx) ** (-float(scheme.pq[n][0])) * float(dt) ** (-float(scheme.pq[n][1])) for n in scheme.names]


def lattice_factors(p, q, dx, dt):
    """Conversion factors X_lattice = X_phys * factor of a quantity with
    scaling (p, q), of its flux and of its source (Alg. 1, Dedimensionalize)."""
    return {"state": dx ** (-p) * dt ** (-q), "flux": dx ** (-(p + 1)) * dt ** (-(q - 1)),
            "source": dx ** (-p) * dt ** (1 - q)}


# --------------------------------------------------------------------------
# Emit: a device functor for the step kernel
# --------------------------------------------------------------------------
class _KernelPrinter(CXX17CodePrinter):
    """C++ for the kernels' arithmetic type: literals as R(...), small
    integer powers as products, square roots through lbm_sqrt."""

    def __init__(self, symbol_map):
        super().__init__()
        self.symbol_map = symbol_map

    def _print_Symbol(self, s):
        return self.symbol_map.get(s, s.name)

    def _print_Integer(self, e):
        return f"R({int(e)})"

    def _print_Rational(self, e):
        return f"(R({e.p}) / R({e.q}))"

    def _print_Float(self, e):
        return f"R({float(e)!r})"

    def _print_Pow(self, e):
        b, x = e.args
        if x == sp.Rational(1, 2):
            return f"lbm_sqrt({self._print(b)})"
        if x == -sp.Rational(1, 2):
            return f"(R(1) / lbm_sqrt({self._print(b)}))"
        if x.is_Integer and 0 < abs(int(x)) <= 8:
            base = self.parenthesize(b, PRECEDENCE["Mul"] + 1)
            prod = " * ".join([base] * abs(int(x)))
            return f"({prod})" if x > 0 else f"(R(1) / ({prod}))"
        raise ValueError(f"unsupported power {e}")


def fluctuation_form(scheme: Scheme):
    """Flux deviations Phi(Q0 + dQ) - Phi(Q0) written so that the reference
    terms cancel symbolically: with Phi = N / M (one rational function per
    component), the deviation is (N(Q0 + dQ) M(Q0) - N(Q0) M(Q0 + dQ)) /
    (M(Q0 + dQ) M(Q0)); the expanded numerator keeps only terms with a dQ
    factor, so no large reference-sized terms cancel in floating point (the
    Automated Reference and Equilibrium Shifting of Sec. 2.5.2, done by the
    compiler).  Tracker references are zero.  Returns (q0, dq, [[delta]])."""
    K = scheme.K
    q0 = [sp.Symbol(f"q0_{k}", real=True) for k in range(K)]
    dq = [sp.Symbol(f"dq_{k}", real=True) for k in range(K)]
    full = {f: (q0[k] + dq[k] if k < scheme.n_conserved else dq[k]) for k, f in enumerate(scheme.fields)}
    ref = {f: (q0[k] if k < scheme.n_conserved else sp.Integer(0)) for k, f in enumerate(scheme.fields)}
    zero_dq = {d: 0 for d in dq}
    out = []
    for row in scheme.flux:
        drow = []
        for e in row:
            N, M = sp.fraction(sp.together(e))
            Nf, Mf = N.xreplace(full), M.xreplace(full)
            N0, M0 = N.xreplace(ref), M.xreplace(ref)
            num = sp.expand(Nf * M0 - N0 * Mf)
            terms = sp.Add.make_args(num)
            keep = [t for t in terms if t.free_symbols & set(dq)]
            rest = sp.expand(sp.Add(*[t for t in terms if not (t.free_symbols & set(dq))]))
            if rest != 0:
                raise ValueError("reference terms did not cancel")
            numr = sp.collect(sp.Add(*keep), dq, evaluate=True)
            drow.append(numr / (Mf * M0) if M != 1 else numr)
        out.append(drow)
    return q0, dq, out


def emit_functor(scheme: Scheme, struct: str, sys_id: int) -> str:
    """C++ source of a system functor with the interface of the library's
    hand-written systems (K, D, id, tracker(), flux_delta, source,
    max_speed).  flux_delta evaluates the compiler's fluctuation form of the
    flux (``fluctuation_form``), source the declared source at the absolute
    state.  Parameters are read from the kernel parameter block's generic
    slots, 1/tau_grad from its tracker slot, Q0 from the reference state."""
    K, D = scheme.K, scheme.dim
    q0, dq, dflux = fluctuation_form(scheme)
    psym = {s: f"p.gen[{j}]" for j, s in enumerate(scheme.params)}
    base = dict(psym)
    base[scheme.inv_tau_grad] = "p.inv_tau_grad"

    def block(exprs, smap, targets):
        merged = dict(base)
        merged.update(smap)
        pr = _KernelPrinter(merged)
        tmps, red = sp.cse(exprs, symbols=sp.numbered_symbols("t"))
        out = []
        for t, e in tmps:
            pr.symbol_map[t] = str(t)
            out.append(f"        const S {t} = {pr.doprint(e)};")
        for tgt, e in zip(targets, red):
            out.append(f"        {tgt} = {pr.doprint(e)};")
        return out

    fsmap = {d: f"dQ[{k}]" for k, d in enumerate(dq)}
    fsmap.update({q: f"p.Q0[{k}]" for k, q in enumerate(q0)})
    flux_lines = block([e for row in dflux for e in row], fsmap,
                       [f"dPhi[{k}][{c}]" for k in range(K) for c in range(D)])
    ssmap = {f: f"Q[{k}]" for k, f in enumerate(scheme.fields)}
    src_lines = block(list(scheme.source), ssmap, [f"Sk[{k}]" for k in range(K)])
    trk = " || ".join(f"k == {k}" for k in range(scheme.n_conserved, K)) or "false"
    lines = [f"// Generated from the declared conservation law '{scheme.name}' (fields: "
             + ", ".join(scheme.names) + ").",
             f"struct {struct} {{",
             f"    static constexpr int K = {K}, D = {D}, id = {sys_id};",
             "    static constexpr bool precise = false;",
             "    static constexpr bool compensated = true;",
             f"    static constexpr bool tracker(int k) {{ return {trk}; }}",
             "",
             "    template <class S, class R>",
             "    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])",
             "    {"] + flux_lines + [
             "    }",
             "",
             "    template <class S, class R>",
             "    __host__ __device__ static void source(const Phys<R> &p, const S *dQ, const R *, S *Sk)",
             "    {",
             "        S Q[K];",
             "#pragma unroll",
             "        for (int k = 0; k < K; ++k) Q[k] = dQ[k] + p.Q0[k];"] + src_lines + [
             "    }",
             "",
             "    // no characteristic speed is derived for generated systems",
             "    template <class R>",
             "    __host__ __device__ static R max_speed(const Phys<R> &, const R *) { return R(0); }",
             "};", ""]
    return "\n".join(lines)
