"""The C-ABI library loads on a machine without a GPU and exports every
function that include/qdpmi.h declares (no compute calls are made here)."""

import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qdpmi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:qdp_status|const char\s*\*)\s*(qdp_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["qdp_init", "qdp_finalize", "qdp_lattice_create", "qdp_field_alloc", "qdp_field_free",
                     "qdp_field_write", "qdp_field_read", "qdp_eval", "qdp_shift", "qdp_sum_multi",
                     "qdp_smear_jacobi", "qdp_smear_jacobi_batch", "qdp_hadron_contract", "qdp_cache_stats",
                     "qdp_cache_evict", "qdp_set_pool_limit", "qdp_sync", "qdp_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1111_5596_amd import qdpmi

    names = declared_functions()
    missing = [n for n in names if not hasattr(qdpmi.lib, n)]
    assert not missing, missing
    assert set(names) == set(qdpmi.SIGNATURES), set(names) ^ set(qdpmi.SIGNATURES)


def test_null_arguments_are_rejected_without_a_device():
    from paper_1111_5596_amd import qdpmi

    assert qdpmi.lib.qdp_init(None, None) == -1
    assert qdpmi.lib.qdp_last_error(None) == b"null context"
    assert qdpmi.lib.qdp_sync(None) == -1


def test_binding_refuses_propagators_without_12_columns():
    """The contraction entry points read exactly 12 column handles; the
    binding refuses any other count before calling the library (no context
    or device is needed to reach the check)."""
    import pytest

    from paper_1111_5596_amd import qdpmi

    ctx = qdpmi.Context.__new__(qdpmi.Context)  # no library context behind it
    eleven, thirteen, twelve = list(range(1, 12)), list(range(1, 14)), list(range(1, 13))
    calls = [lambda S: ctx.contract(S, twelve), lambda S: ctx.contract(twelve, S),
             lambda S: ctx.contract_mom(S, twelve, [(0, 0, 0)]), lambda S: ctx.nucleon(twelve, S),
             lambda S: ctx.nucleon(S, twelve), lambda S: ctx.delta(S)]
    for call in calls:
        for bad in (eleven, thirteen, []):
            with pytest.raises(ValueError, match="12 column handles"):
                call(bad)
    assert len(qdpmi._propagator(twelve, "x")) == 12
