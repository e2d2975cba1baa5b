"""The phase counter of the descent kernel's assembly reads the compiler's
loop comments: a small hand-written function with the descent kernel's loop
nest (iteration loop holding a forward-step loop and a segment loop with a
recompute and a reverse loop) must be split into the right phases."""
from paper_1704_02524_amd import isa_phases as I

ASM = """\
fn:
\ts_load_dwordx2 s[0:1], s[4:5], 0x0
.LBB0_1:                                ; =>This Loop Header: Depth=1
                                        ;     Child Loop BB0_2 Depth 2
                                        ;     Child Loop BB0_3 Depth 2
\tv_mov_b32 v0, 0
.LBB0_2:                                ;   Parent Loop BB0_1 Depth=1
                                        ; =>  This Inner Loop Header: Depth=2
\tv_fma_f64 v[0:1], v[2:3], v[4:5], v[0:1]
\tv_fma_f64 v[0:1], v[2:3], v[4:5], v[0:1]
\tglobal_store_dwordx2 v[6:7], v[0:1], off
\ts_cbranch_scc0 .LBB0_2
; %bb.5:                                ;   in Loop: Header=BB0_1 Depth=1
\tv_add_f64 v[0:1], v[0:1], v[2:3]
.LBB0_3:                                ;   Parent Loop BB0_1 Depth=1
                                        ; =>  This Loop Header: Depth=2
                                        ;       Child Loop BB0_4 Depth 3
                                        ;       Child Loop BB0_6 Depth 3
\ts_mov_b32 s2, 0
.LBB0_4:                                ;   Parent Loop BB0_1 Depth=1
                                        ;     Parent Loop BB0_3 Depth=2
                                        ; =>    This Inner Loop Header: Depth=3
\tv_mul_f64 v[0:1], v[0:1], v[2:3]
\tds_write_b64 v8, v[0:1]
\ts_cbranch_scc0 .LBB0_4
.LBB0_6:                                ;   Parent Loop BB0_1 Depth=1
                                        ;     Parent Loop BB0_3 Depth=2
                                        ; =>    This Inner Loop Header: Depth=3
\tv_accvgpr_read_b32 v9, a0
\tv_fma_f64 v[0:1], v[2:3], v[4:5], v[0:1]
\tv_fma_f64 v[0:1], v[2:3], v[4:5], v[0:1]
\tv_fma_f64 v[0:1], v[2:3], v[4:5], v[0:1]
\tv_cndmask_b32 v9, v9, v10, vcc
\ts_cbranch_scc0 .LBB0_6
; %bb.7:                                ;   in Loop: Header=BB0_3 Depth=2
\ts_cbranch_scc0 .LBB0_3
; %bb.8:                                ;   in Loop: Header=BB0_1 Depth=1
\ts_cbranch_scc0 .LBB0_1
; %bb.9:
\ts_endpgm
.Lfunc_end0:
"""


def test_loop_nest_is_split_into_the_three_phases(tmp_path):
    p = tmp_path / "k.s"
    p.write_text(ASM)
    blocks, loops = I.parse(str(p), "fn")
    assert loops["BB0_4"]["parent"] == "BB0_3" and loops["BB0_3"]["parent"] == "BB0_1"
    ph = I.phases(blocks, loops)
    assert ph["forward"] == {"fp64": 2, "global": 1, "salu": 1, "steps_per_pass": 1}
    assert ph["recompute"] == {"fp64": 1, "lds": 1, "salu": 1, "steps_per_pass": 1}
    assert ph["reverse"] == {"agpr": 1, "fp64": 3, "valu_other": 1, "salu": 1,
                             "steps_per_pass": 1}


def test_unrolled_loop_bodies_are_counted_per_step(tmp_path):
    """Eight hardware reciprocals (two steps of four tanh) in the forward
    loop: its counts are halved."""
    rcp = "\tv_rcp_f64_e32 v[0:1], v[2:3]\n"
    p = tmp_path / "k.s"
    p.write_text(ASM.replace("\tglobal_store_dwordx2", rcp * 8 + "\tglobal_store_dwordx2"))
    blocks, loops = I.parse(str(p), "fn")
    ph = I.phases(blocks, loops, tanh_steps=True)
    assert ph["forward"]["steps_per_pass"] == 2
    assert ph["forward"]["fp64"] == (2 + 8) / 2


def test_kernel_symbol_names_the_single_instance_adjoint_descent():
    s = I.kernel_symbol(10, 1, 2)
    assert s.startswith("_ZN2hj10k_solve_gd") and "CfgIdLi10ELi1ELi2E" in s
    assert "ELi0EEEv" in s and "ELi2EEEv" in I.kernel_symbol(5, 2, 2, 2)
