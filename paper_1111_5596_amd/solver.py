"""Solver algebra written in lattice-field expressions.

The paper's QUDA integration (QUDA-integration subsection) lets the
propagator solve and the expression layer share one device pool, and has the
residual calculation and solution reconstruction run as expressions.  This
module is that algebra for the operator the smearing applies, M = 1 + kappa H
(H the gauge-covariant spatial hopping term of the smearing step): a
conjugate-gradient solve of M x = b where every field operation is a qdp_eval
(the operator as one fused stencil expression, axpy updates) and every inner
product a qdp_sum_multi (FP64 sums).  M is Hermitian (H is), and positive
definite for |kappa| < 1/6 since the spectrum of H lies in [-6, 6].

Nothing here touches field data on the host: the loop only moves the scalars
alpha, beta and the residual norms.
"""

from __future__ import annotations


def jacobi_program(gauge, src, kappa):
    """Postfix program of (1 + kappa H) src, spatial directions 0..2."""
    prog = [("field", src)]
    for i in range(3):
        prog += [("gauge", gauge, i), ("field", src), ("shift", i, 1), ("mul",),
                 ("real_const", kappa), ("mul",), ("add",)]
        prog += [("gauge", gauge, i), ("adj",), ("field", src), ("mul",), ("shift", i, -1),
                 ("real_const", kappa), ("mul",), ("add",)]
    return prog


def norm2(q, f) -> float:
    """Global sum of |f(x)|^2 in FP64."""
    return float(q.sum_multi([("field", f), ("local_norm2",)])[0, 0].real)


def inner(q, a, b) -> complex:
    """Global sum of a(x)^dagger b(x) in FP64."""
    return complex(q.sum_multi([("field", a), ("field", b), ("local_inner",)])[0, 0])


def cg_jacobi(q, gauge, b, x, kappa, tol=1e-10, maxiter=500):
    """Solve (1 + kappa H) x = b by conjugate gradient, x holding the start
    vector on entry and the solution on exit.  Returns (iterations, true
    relative residual |b - M x| / |b|, recomputed from x at the end).

    Fields: b, x FERMION of one lattice and precision; gauge the links of that
    lattice.  Three work fields of the same kind are taken from the pool."""
    if not abs(kappa) < 1.0 / 6.0:
        raise ValueError("1 + kappa H is positive definite only for |kappa| < 1/6")
    lat, t, prec = q.field_meta[x]
    r, p, ap = (q.alloc(lat, t, prec) for _ in range(3))
    try:
        bb = norm2(q, b)
        if bb == 0.0:
            q.eval([("field", b)], x)
            return 0, 0.0
        q.eval(jacobi_program(gauge, x, kappa), ap)
        q.eval([("field", b), ("field", ap), ("sub",)], r)
        q.eval([("field", r)], p)
        rr = norm2(q, r)
        it = 0
        while it < maxiter and rr > tol * tol * bb:
            q.eval(jacobi_program(gauge, p, kappa), ap)
            alpha = rr / inner(q, p, ap).real
            q.eval([("field", p), ("real_const", alpha), ("mul",)], x, assign="+=")
            q.eval([("field", ap), ("real_const", alpha), ("mul",)], r, assign="-=")
            rr_new = norm2(q, r)
            beta = rr_new / rr
            q.eval([("field", r), ("field", p), ("real_const", beta), ("mul",), ("add",)], p)
            rr = rr_new
            it += 1
        # solution check: the true residual, not the recursively updated one
        q.eval(jacobi_program(gauge, x, kappa), ap)
        q.eval([("field", b), ("field", ap), ("sub",)], r)
        return it, (norm2(q, r) / bb) ** 0.5
    finally:
        for f in (r, p, ap):
            q.free(f)
