"""C-ABI checks that need no GPU: the library loads, exports every entry point
the header declares, and host-only validation behaves as documented."""
import ctypes
import os
import re

import pytest

from paper_1810_01609_amd import mdwf as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdwf.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"MDWF_API\s+[\w\s\*]*?\b(mdwf_\w+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    lib = M.lib()
    for n in names:
        assert hasattr(lib, n), f"{n} declared in mdwf.h but not exported"
    # the binding declares a signature for each of them
    assert set(names) <= set(M._SIGS), set(names) - set(M._SIGS)


def test_abi_version():
    assert M.lib().mdwf_abi_version() == 1


@pytest.mark.parametrize(
    "kw,frag",
    [
        (dict(L=(3, 4, 4, 4), L5=4), "Lx must be even"),
        (dict(L=(4, 1, 4, 4), L5=4), "Ly must be >= 2"),
        (dict(L=(4, 4, 4, 4), L5=0), "L5 must be in"),
        (dict(L=(4, 4, 4, 4), L5=33), "L5 must be in"),
        (dict(L=(4, 4, 4, 4), L5=4, mq=-0.1), "mq must be >= 0"),
        (dict(L=(4, 4, 4, 4), L5=4, b5=float("nan")), "finite"),
        (dict(L=(4, 4, 4, 4), L5=4, t_antiperiodic=2), "t_antiperiodic"),
    ],
)
def test_check_action_rejects(kw, frag):
    act = M.Action.make(**kw)
    st, msg = M.check_action(act)
    assert st == M.EINVAL
    assert frag in msg


def test_check_action_accepts_benchmark_configs():
    import mdwf_synth as S

    for name, c in S.CONFIGS.items():
        act = M.Action.make(c["L"], c["L5"], c["b5"], c["c5"], c["M5"], c["mq"])
        assert M.check_action(act) == (M.OK, ""), name


def test_job_footprint_model():
    act = M.Action.make((32, 32, 32, 64), 12, mq=0.005)
    Vh = 32 * 32 * 32 * 64 // 2
    ne = Vh * 12
    f64 = M.job_footprint(act, M.CGOpts.make(inner="f64"), 1)
    f32 = M.job_footprint(act, M.CGOpts.make(inner="f32"), 12)
    f16 = M.job_footprint(act, M.CGOpts.make(inner="f16"), 12)
    # FP64: r p M_phi p t v x eta^ (7 fields) + 3 context temporaries
    assert f64 >= 10 * ne * 192
    # FP32 per RHS: 5 FP32 work fields (r, p, M_phi p, t, v) + FP32 x + FP64 xh + FP64 eta^
    assert f32 >= 12 * (6 * ne * 96 + 2 * ne * 192) + 3 * ne * 192
    assert f32 < 12 * (6 * ne * 96 + 2 * ne * 192) + 3 * ne * 192 + 64 * 1024
    assert f16 < f32
    assert M.job_footprint(act, M.CGOpts.make(inner="f64"), 0) == 0


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(M, "_lib", None)
    monkeypatch.setattr(M, "LIB_PATH", "/nonexistent/libmdwf.so")
    with pytest.raises(M.MDWFError):
        M.lib()


def test_ended_job_drops_its_tensor_references():
    """Job keeps the source and solution tensors alive only while the job
    runs: end() drops them even if the Job object itself stays referenced
    (here a job whose handle was already released, so no device call is made)."""
    import weakref

    class Buf:  # stands in for a tensor
        pass

    eta, psi = Buf(), Buf()
    refs = [weakref.ref(eta), weakref.ref(psi)]
    job = M.Job(None, ctypes.c_void_p(), 2, keep=(eta, psi))
    del eta, psi
    assert all(r() is not None for r in refs)
    job.end()
    assert all(r() is None for r in refs)
