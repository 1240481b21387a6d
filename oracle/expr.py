"""Plain numpy evaluator of site-local lattice expressions (test infrastructure).

This is the oracle for expression evaluation (the paper's section 4.2: a
single expression ``dest = expr`` over lattice objects, evaluated site by
site; QDP++ semantics for the operations).  Everything is complex128.

A program is a postfix list of tuples.  Leaves push a value, operators pop
their operands (binary operators pop the right operand first):

    ('field', key)            field from the ``fields`` dict: (type, array)
    ('gauge', key, mu)        colour matrix U_mu of a gauge field (4, V, 3, 3)
    ('real_const', x)         REAL constant
    ('complex_const', re, im) COMPLEX constant
    ('shift', mu, sign)       value(x + sign * mu_hat), periodic
    ('neg',) ('conj',) ('adj',)
    ('add',) ('sub',) ('mul',)
    ('gamma_left', n) ('gamma_right', n)   Gamma_n * a,  a * Gamma_n
    ('trace',) ('trace_color',) ('trace_spin',)
    ('real',) ('imag',) ('local_norm2',) ('local_inner',)

Types and their per-site index shapes (spin_row, spin_col, colour_row,
colour_col); canonical host arrays drop the unit axes:

    REAL (1,1,1,1)  COMPLEX (1,1,1,1)  COLOR_VECTOR (1,1,3,1)
    COLOR_MATRIX (1,1,3,3)  FERMION (4,1,3,1)  SPIN_MATRIX (4,4,1,1)
    PROPAGATOR (4,4,3,3)

A product multiplies the spin parts and the colour parts as matrices; an
operand whose spin (or colour) part is a scalar acts as the identity there.
"""

from __future__ import annotations

import numpy as np

from . import gamma as _gamma

SHAPES = {
    "REAL": (1, 1, 1, 1),
    "COMPLEX": (1, 1, 1, 1),
    "COLOR_VECTOR": (1, 1, 3, 1),
    "COLOR_MATRIX": (1, 1, 3, 3),
    "FERMION": (4, 1, 3, 1),
    "SPIN_MATRIX": (4, 4, 1, 1),
    "PROPAGATOR": (4, 4, 3, 3),
}
CANONICAL = {
    "REAL": (),
    "COMPLEX": (),
    "COLOR_VECTOR": (3,),
    "COLOR_MATRIX": (3, 3),
    "FERMION": (4, 3),
    "SPIN_MATRIX": (4, 4),
    "PROPAGATOR": (4, 4, 3, 3),
}


class ExprTypeError(ValueError):
    pass


def _type_of_shape(shape, real: bool) -> str:
    if shape == (1, 1, 1, 1):
        return "REAL" if real else "COMPLEX"
    for name, s in SHAPES.items():
        if s == shape and name not in ("REAL", "COMPLEX"):
            return name
    raise ExprTypeError(f"no lattice type has site shape {shape}")


def to_generic(type_name: str, arr: np.ndarray) -> np.ndarray:
    a = np.asarray(arr, dtype=np.complex128)
    return a.reshape((a.shape[0],) + SHAPES[type_name])


def to_canonical(type_name: str, arr: np.ndarray) -> np.ndarray:
    out = arr.reshape((arr.shape[0],) + CANONICAL[type_name])
    if type_name == "REAL":
        return out.real.copy()
    return out


def _roll(dims, arr, mu, sign):
    """value(x + sign*mu_hat): roll the lattice axes of a (V, ...) array."""
    Lx, Ly, Lz, Lt = dims
    rest = arr.shape[1:]
    a = arr.reshape((Lt, Lz, Ly, Lx) + rest)
    axis = 3 - mu  # x is the last lattice axis
    return np.roll(a, -sign, axis=axis).reshape(arr.shape)


def _expand(a, part, n):
    """Replace a scalar spin (part=0) or colour (part=1) factor by identity(n)."""
    eye = np.eye(n, dtype=np.complex128)
    if part == 0:
        return a[:, 0, 0, None, None, :, :] * eye[None, :, :, None, None]
    return a[:, :, :, 0, 0, None, None] * eye[None, None, None, :, :]


def _mul(ta, a, tb, b):
    sa, sb = a.shape[1:], b.shape[1:]
    # spin part
    if sa[:2] == (1, 1) and sb[:2] != (1, 1):
        a = _expand(a, 0, sb[0])
    elif sb[:2] == (1, 1) and sa[:2] != (1, 1):
        b = _expand(b, 0, sa[1])
    sa, sb = a.shape[1:], b.shape[1:]
    if sa[2:] == (1, 1) and sb[2:] != (1, 1):
        a = _expand(a, 1, sb[2])
    elif sb[2:] == (1, 1) and sa[2:] != (1, 1):
        b = _expand(b, 1, sa[3])
    sa, sb = a.shape[1:], b.shape[1:]
    if sa[1] != sb[0] or sa[3] != sb[2]:
        raise ExprTypeError(f"cannot multiply {ta} by {tb}")
    out = np.einsum("vijab,vjkbc->vikac", a, b)
    return _type_of_shape(out.shape[1:], ta == "REAL" and tb == "REAL"), out


def _add(ta, a, tb, b, sign):
    if ta != tb:
        scalars = {"REAL", "COMPLEX"}
        if not (ta in scalars and tb in scalars):
            raise ExprTypeError(f"cannot add {ta} and {tb}")
        t = "COMPLEX"
    else:
        t = ta
    return t, a + sign * b


def _gamma_left(n, t, a):
    if a.shape[1] != 4:
        raise ExprTypeError(f"Gamma * {t}: no spin row index")
    g = _gamma(n)
    return t, np.einsum("ij,vjkab->vikab", g, a)


def _gamma_right(n, t, a):
    if a.shape[2] != 4:
        raise ExprTypeError(f"{t} * Gamma: no spin column index")
    g = _gamma(n)
    return t, np.einsum("vijab,jk->vikab", a, g)


def _adj(t, a):
    s = a.shape[1:]
    if (s[0] != s[1]) or (s[2] != s[3]):
        raise ExprTypeError(f"adj of {t}")
    return t, np.conj(np.transpose(a, (0, 2, 1, 4, 3)))


def _trace(t, a):
    if t not in ("REAL", "COMPLEX", "COLOR_MATRIX", "SPIN_MATRIX", "PROPAGATOR"):
        raise ExprTypeError(f"trace of {t}")
    v = np.einsum("viiaa->v", a)
    return ("REAL" if t == "REAL" else "COMPLEX"), v.reshape(-1, 1, 1, 1, 1)


def _trace_color(t, a):
    if t not in ("COLOR_MATRIX", "PROPAGATOR"):
        raise ExprTypeError(f"traceColor of {t}")
    v = np.einsum("vijaa->vij", a)[:, :, :, None, None]
    return _type_of_shape(v.shape[1:], False), v


def _trace_spin(t, a):
    if t not in ("SPIN_MATRIX", "PROPAGATOR"):
        raise ExprTypeError(f"traceSpin of {t}")
    v = np.einsum("viiab->vab", a)[:, None, None, :, :]
    return _type_of_shape(v.shape[1:], False), v


def evaluate(program, fields, dims):
    """Evaluate a postfix program at every site; returns (type, generic array)."""
    V = int(np.prod(dims))
    stack = []
    for node in program:
        op = node[0]
        if op == "field":
            t, arr = fields[node[1]]
            stack.append((t, to_generic(t, arr)))
        elif op == "gauge":
            _, arr = fields[node[1]]
            stack.append(("COLOR_MATRIX", to_generic("COLOR_MATRIX", np.asarray(arr)[node[2]])))
        elif op == "real_const":
            stack.append(("REAL", np.full((V, 1, 1, 1, 1), complex(node[1], 0.0))))
        elif op == "complex_const":
            stack.append(("COMPLEX", np.full((V, 1, 1, 1, 1), complex(node[1], node[2]))))
        elif op == "shift":
            t, a = stack.pop()
            stack.append((t, _roll(dims, a, node[1], node[2])))
        elif op == "neg":
            t, a = stack.pop()
            stack.append((t, -a))
        elif op == "conj":
            t, a = stack.pop()
            stack.append((t, np.conj(a)))
        elif op == "adj":
            stack.append(_adj(*stack.pop()))
        elif op in ("add", "sub", "mul", "local_inner"):
            tb, b = stack.pop()
            ta, a = stack.pop()
            if op == "add":
                stack.append(_add(ta, a, tb, b, 1.0))
            elif op == "sub":
                stack.append(_add(ta, a, tb, b, -1.0))
            elif op == "mul":
                stack.append(_mul(ta, a, tb, b))
            else:
                if a.shape != b.shape:
                    raise ExprTypeError(f"localInnerProduct of {ta} and {tb}")
                v = np.sum(np.conj(a) * b, axis=(1, 2, 3, 4))
                stack.append(("COMPLEX", v.reshape(-1, 1, 1, 1, 1)))
        elif op == "gamma_left":
            stack.append(_gamma_left(node[1], *stack.pop()))
        elif op == "gamma_right":
            stack.append(_gamma_right(node[1], *stack.pop()))
        elif op == "trace":
            stack.append(_trace(*stack.pop()))
        elif op == "trace_color":
            stack.append(_trace_color(*stack.pop()))
        elif op == "trace_spin":
            stack.append(_trace_spin(*stack.pop()))
        elif op in ("real", "imag"):
            t, a = stack.pop()
            if t not in ("REAL", "COMPLEX"):
                raise ExprTypeError(f"{op} of {t}")
            v = a.real if op == "real" else a.imag
            stack.append(("REAL", v.astype(np.complex128)))
        elif op == "local_norm2":
            t, a = stack.pop()
            v = np.sum(np.abs(a) ** 2, axis=(1, 2, 3, 4))
            stack.append(("REAL", v.astype(np.complex128).reshape(-1, 1, 1, 1, 1)))
        else:
            raise ExprTypeError(f"unknown op {op}")
    if len(stack) != 1:
        raise ExprTypeError("malformed program")
    return stack[0]


def subset_mask(dims, subset) -> np.ndarray:
    """Boolean mask over lexicographic sites: 'all', 'even', 'odd' or
    ('timeslice', t).  Parity is (x + y + z + t) mod 2."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    if subset == "all":
        m = np.ones_like(x, dtype=bool)
    elif subset == "even":
        m = (x + y + z + t) % 2 == 0
    elif subset == "odd":
        m = (x + y + z + t) % 2 == 1
    else:
        kind, tt = subset
        assert kind == "timeslice"
        m = t == tt
    return m.reshape(-1)


def assign(program, fields, dims, dest_type, dest, subset="all", op="="):
    """QDP assignment ``dest op= expr`` over a subset; other sites unchanged.

    Returns the new canonical dest array."""
    t, val = evaluate(program, fields, dims)
    d = to_generic(dest_type, dest).copy()
    if op == "*=":
        t, val = _mul(dest_type, d, t, val)
    if t != dest_type and not (t == "REAL" and dest_type == "COMPLEX"):
        raise ExprTypeError(f"cannot assign {t} to {dest_type}")
    m = subset_mask(dims, subset)
    if op == "=" or op == "*=":
        d[m] = val[m]
    elif op == "+=":
        d[m] = d[m] + val[m]
    elif op == "-=":
        d[m] = d[m] - val[m]
    else:
        raise ValueError(op)
    return to_canonical(dest_type, d)


def sum_multi(program, fields, dims, kind):
    """Sums of every component of expr over the subsets of a set, FP64.

    kind: 'all' (1 subset), 'parity' (even, odd) or 'timeslice' (Lt subsets).
    Returns an (nsub, ncomp) complex array, summed in lexicographic order."""
    t, val = evaluate(program, fields, dims)
    flat = val.reshape(val.shape[0], -1)
    if kind == "all":
        masks = [subset_mask(dims, "all")]
    elif kind == "parity":
        masks = [subset_mask(dims, "even"), subset_mask(dims, "odd")]
    else:
        masks = [subset_mask(dims, ("timeslice", tt)) for tt in range(dims[3])]
    out = np.zeros((len(masks), flat.shape[1]), dtype=np.complex128)
    for i, m in enumerate(masks):
        sel = flat[m]
        if sel.shape[0]:
            # cumulative sum = strictly sequential order over the sites
            out[i] = np.cumsum(sel, axis=0)[-1]
    return t, out
