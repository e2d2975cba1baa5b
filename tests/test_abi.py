"""Host-only checks of the C interface: the library loads, exports every
function declared in include/hj.h, and rejects bad arguments before any
device work (so these run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hj.h")
LIB = os.path.join(ROOT, "paper_1704_02524_amd", "libhj.so")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int32_t|size_t|const char \*)\s*(hj_\w+)\s*\(", txt,
                                 re.M)))


def _need_lib():
    if not os.path.exists(LIB):
        from paper_1704_02524_amd import build
        build.build()


def test_header_declares_the_entry_points():
    assert set(_declared()) >= {"hj_solve", "hj_eval", "hj_workspace_size", "hj_last_error",
                                "hj_version"}


def test_library_exports_every_declared_symbol():
    _need_lib()
    L = C.CDLL(LIB)
    for name in _declared():
        assert hasattr(L, name), name
    L.hj_version.restype = C.c_int32
    assert L.hj_version() == 1


def _wl():
    from paper_1704_02524_amd import workloads as W
    return W.c1_hopf_n10(B=2)


def _call_solve(wl, B=2, n=None, t=None, nsteps=None, G=4, R=2, xptr=1, entry="hj_solve",
                **opt):
    from paper_1704_02524_amd import hj
    L = hj.lib()
    prob = hj.Problem(wl)
    o = hj.Opts()
    for k, v in dict(dtype=0, formula=1, mode=1, quad=1, max_iter=10, ckpt_K=16, cert_fp64=1,
                     alpha0=0.3, fd_sigma=1e-4, eps_step=1e-10, cert_tol=1e-8, v_max=1e6,
                     acc_rel=1e-14).items():
        setattr(o, k, v)
    for k, v in opt.items():
        setattr(o, k, v)
    gs = hj.Guesses(G, R, C.c_void_p(1))
    rc = getattr(L, entry)(0, C.byref(prob.H), 0, C.byref(prob.J), C.c_void_p(xptr), B,
                    wl.n if n is None else n, wl.t if t is None else t,
                    wl.nsteps if nsteps is None else nsteps, C.byref(gs), C.byref(o),
                    C.c_void_p(1), C.c_void_p(1), C.c_void_p(1), None)
    return rc, L.hj_last_error().decode()


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), -1), (dict(n=200), -5), (dict(t=0.0), -1), (dict(t=-1.0), -1),
    (dict(t=float("nan")), -1), (dict(nsteps=0), -1), (dict(G=0), -1), (dict(G=65), -1),
    (dict(R=-1), -1), (dict(B=-3), -1), (dict(dtype=7), -2), (dict(mode=5), -1),
    (dict(quad=9), -1), (dict(max_iter=-1), -1), (dict(ckpt_K=0), -1), (dict(alpha0=0.0), -1),
])
@pytest.mark.parametrize("entry", ["hj_solve", "hj_solve_noalloc"])
def test_invalid_arguments_are_rejected(kw, code, entry):
    rc, msg = _call_solve(_wl(), entry=entry, **kw)
    assert rc == code
    assert msg


def test_noalloc_entry_point_refuses_a_caller_workspace():
    """hj_solve_noalloc works in the library's fixed scratch only."""
    rc, msg = _call_solve(_wl(), entry="hj_solve_noalloc", workspace=C.c_void_p(4096),
                          ws_bytes=1 << 20)
    assert rc == -1 and "workspace" in msg
    rc, msg = _call_solve(_wl(), B=0, xptr=0, entry="hj_solve_noalloc")
    assert rc == 0 and msg == ""


def test_zero_points_is_a_noop():
    rc, msg = _call_solve(_wl(), B=0, xptr=0)
    assert rc == 0 and msg == ""


def test_unknown_kinds_and_drift_are_reported():
    from paper_1704_02524_amd import hj
    wl = _wl()
    L = hj.lib()
    prob = hj.Problem(wl)
    gs = hj.Guesses(4, 2, C.c_void_p(1))
    rc = L.hj_solve(3, C.byref(prob.H), 0, C.byref(prob.J), C.c_void_p(1), 2, wl.n, wl.t,
                    wl.nsteps, C.byref(gs), None, C.c_void_p(1), C.c_void_p(1),
                    C.c_void_p(1), None)
    assert rc == -5
    bad_a = np.array(wl.a)
    bad_a[3] = 0.0
    prob2 = hj.Problem(wl.with_(a=bad_a))
    rc = L.hj_solve(0, C.byref(prob2.H), 0, C.byref(prob2.J), C.c_void_p(1), 2, wl.n, wl.t,
                    wl.nsteps, C.byref(gs), None, C.c_void_p(1), C.c_void_p(1),
                    C.c_void_p(1), None)
    assert rc == -1


def test_workspace_size_grows_with_the_problem():
    from paper_1704_02524_amd import hj
    L = hj.lib()
    small = L.hj_workspace_size(10, 16, 4, 128, None)
    big = L.hj_workspace_size(10, 4096, 16, 128, None)
    assert 0 < small < big
    assert L.hj_workspace_size(0, 16, 4, 128, None) == 0


def test_drift_limits_are_reported():
    """The linear-drift kernels run on the matrix-core layout (4 lanes per
    task, n <= 64); other requests and non-finite drift entries are errors
    raised before any device work."""
    from paper_1704_02524_amd import workloads as W
    wl = W.c3_drift_n32(B=2)
    rc, msg = _call_solve(wl, lanes_per_task=2)
    assert rc == -5 and "drift" in msg
    big = W.c3_drift_n32(B=2).with_(n=65, A=np.eye(65) * 0.5, d=np.ones(65), a=np.ones(65),
                                    x=np.zeros((2, 65)))
    rc, msg = _call_solve(big)
    assert rc == -5 and "drift" in msg
    A = wl.A.copy()
    A[3, 4] = np.inf
    rc, msg = _call_solve(wl.with_(A=A))
    assert rc == -1 and "finite" in msg


def test_device_code_keeps_fp32_arithmetic_in_fp32():
    """Device code takes fused multiply-adds through the precision-matched
    helper: the bare builtin is the double one, and on float operands it
    converts to double and back around an FP64 FMA (it used to make two
    thirds of the FP32 kernels' instructions conversions and FP64 FMAs)."""
    import os
    import re
    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1704_02524_amd", "csrc")
    for name in ("hj_device.hpp", "hj_kernels.hpp"):
        with open(os.path.join(csrc, name)) as f:
            code = f.read()
        uses = [m.start() for m in re.finditer(r"__builtin_fma\(", code)]
        helper = code.find("__device__ __forceinline__ double fmaT(")
        # the only bare use is inside the double overload of the helper
        assert all(0 <= helper < u < helper + 200 for u in uses), (name, len(uses))


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the C structs have the header's sizes and field
    offsets (a field added on one side only would shift every later one)."""
    import ctypes
    import subprocess
    from paper_1704_02524_amd import hj
    checks = {"hj_opts": (hj.Opts, ["dtype", "stream", "momentum", "group_cfg",
                                    "cont_lanes_per_task", "tail_budget",
                                    "tail_lanes_per_task"]),
              "hj_group_cfg": (hj.GroupCfg, ["n_max", "cont_lanes_per_task"])}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "hj.h"', "int main(void) {"]
    for cname, (_, fields) in checks.items():
        src.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f in fields:
            src.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src += ["  return 0;", "}"]
    c = tmp_path / "sizes.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "sizes"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.check_call(["gcc", "-std=c11", "-I" + os.path.join(root, "include"), str(c),
                           "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).split("\n")
               if line)
    for cname, (cls, fields) in checks.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f in fields:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, f"{cname}.{f}"
