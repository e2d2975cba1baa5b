"""Instructions per step of each phase of a compiled descent kernel.

Compiles one kernel-instantiation source to gfx950 assembly with the
library's own flags (build.py), finds the adjoint descent kernel of the
requested lane shape and reads its loop nest from the loop comments the
compiler writes beside each basic block:

  descent iteration loop
    forward solve:  one RK4 step (+ quadrature, checkpoint store) per pass
    adjoint sweep:  one segment per pass, holding
      recompute:    one RK4 step of the segment from its checkpoint
      reverse:      one reverse RK4 step (stage vector-Jacobian products)

and counts the instructions of each phase's loop body by class (FP64
arithmetic, AGPR moves, other vector, scalar, LDS, global and scratch
memory).  Blocks a pass may skip (the checkpoint store of every K-th
forward step, rare branches) are included, so the counts are those of the
longest pass.  Multiplied by the steps a launch executes per phase, they
trace the executed instructions of the launch to its phases.

    python -m paper_1704_02524_amd.isa_phases --source hj_inst_f64_1.hip \
        --npl 10 --lpt 1 --mk 2 [--tail-source hj_inst_r64_1.hip --tail-npl 5 \
        --tail-lpt 2] [--markdown out.md]
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import re
import subprocess

from paper_1704_02524_amd import build as B

CLASSES = ("fp64", "agpr", "valu_other", "salu", "lds", "global", "scratch", "other")


def op_class(op: str) -> str:
    if op.startswith("v_accvgpr"):
        return "agpr"
    if op.startswith("v_") and "_f64" in op:
        return "fp64"
    if op.startswith("v_"):
        return "valu_other"
    if op.startswith("s_"):
        return "salu"
    if op.startswith("ds_"):
        return "lds"
    if op.startswith(("global_", "buffer_", "flat_")):
        return "global"
    if op.startswith("scratch_"):
        return "scratch"
    return "other"


def assemble(source: str) -> str:
    """gfx950 device assembly of one instantiation source (library flags)."""
    os.makedirs(B.BUILD, exist_ok=True)
    out = os.path.join(B.BUILD, os.path.splitext(source)[0] + ".s")
    cmd = [B.HIPCC, *B.FLAGS, *B.PER_SOURCE.get(source, []), "--cuda-device-only", "-S",
           os.path.join(B.CSRC, source), "-o", out]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    return out


def kernel_symbol(npl: int, lpt: int, mk: int, tail: int = 0) -> str:
    """Mangled name of k_solve_gd for one instance, double, no drift: the
    plain descent (tail 0), the descent with a tail hand-off (1) or the
    continuation of the hand-off (2)."""
    return (f"_ZN2hj10k_solve_gdINS_3CfgIdLi{npl}ELi{lpt}ELi{mk}ELb0ELb0EEELb0ELi{tail}EEEv"
            "NS_9SolveArgsINT_1TEEE")


def parse(asm_path: str, symbol: str):
    """Basic blocks of one function: label, innermost loop header, the loop
    tree (header -> parent, depth), instruction classes per block."""
    lines = open(asm_path).read().split("\n")
    start = next(i for i, l in enumerate(lines) if l.startswith(symbol + ":"))
    end = next(i for i in range(start, len(lines)) if lines[i].strip().startswith(".Lfunc_end"))
    blocks, loops = [], {}
    cur = {"label": "entry", "loop": None, "ops": []}
    i = start + 1
    while i < end:
        line = lines[i]
        m = re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):?(.*)$", line)
        if m:
            blocks.append(cur)
            label = m.group(1).lstrip(".").replace("LBB", "BB")
            comments = [m.group(2)]
            while i + 1 < end and lines[i + 1].strip().startswith(";"):
                i += 1
                comments.append(lines[i])
            text = " ".join(comments)
            loop = None
            h = re.search(r"Loop Header: Depth=(\d+)", text)
            if h:
                parents = re.findall(r"Parent Loop (BB\d+_\d+) Depth=\d+", text)
                loops[label] = {"parent": parents[-1] if parents else None,
                                "depth": int(h.group(1))}
                loop = label
            else:
                h = re.search(r"in Loop: Header=(BB\d+_\d+) Depth=(\d+)", text)
                if h:
                    loop = h.group(1)
            cur = {"label": label, "loop": loop, "ops": []}
        else:
            s = line.strip()
            if s and not s.startswith((";", ".")):
                cur["ops"].append(s.split()[0])
        i += 1
    blocks.append(cur)
    return blocks, loops


def phases(blocks, loops, tanh_steps: bool = False):
    """The forward, recompute and reverse loops of the descent kernel.  With
    tanh_steps (the tanh speed profile: four FP64 tanh per RK4 step in every
    phase, each with one hardware reciprocal), a loop body holding k x 4
    reciprocals is taken as k steps unrolled, and its counts are divided by
    k ("steps_per_pass" records k)."""
    own = collections.defaultdict(collections.Counter)
    rcp = collections.Counter()
    order = []
    for b in blocks:
        if b["loop"]:
            if b["loop"] not in order:
                order.append(b["loop"])
            own[b["loop"]].update(op_class(op) for op in b["ops"])
            rcp[b["loop"]] += sum(op.startswith("v_rcp_f64") for op in b["ops"])
    children = collections.defaultdict(list)
    for h, info in loops.items():
        if info["parent"]:
            children[info["parent"]].append(h)
    # the descent iteration loop: the outermost loop holding the most code
    top = max((h for h in loops if loops[h]["depth"] == 1),
              key=lambda h: sum(sum(own[c].values()) for c in _subtree(h, children)))
    inner = [h for h in order if loops.get(h, {}).get("parent") == top]
    seg = [h for h in inner if children[h]]
    leaf = [h for h in inner if not children[h]]
    if len(seg) != 1 or not leaf:
        raise RuntimeError("unexpected loop nest: %s" % {h: loops[h] for h in loops})
    fwd = max(leaf, key=lambda h: own[h]["fp64"])
    rec, rev = [h for h in order if h in children[seg[0]]][:2]
    out = {}
    for name, h in (("forward", fwd), ("recompute", rec), ("reverse", rev)):
        k = max(1, round(rcp[h] / 4)) if tanh_steps else 1
        c = collections.Counter({key: v / k for key, v in own[h].items()})
        c["steps_per_pass"] = k
        out[name] = c
    return out


def _subtree(h, children):
    out = [h]
    for c in children[h]:
        out += _subtree(c, children)
    return out


def count(source: str, npl: int, lpt: int, mk: int, tail: int = 0) -> dict:
    asm = assemble(source)
    blocks, loops = parse(asm, kernel_symbol(npl, lpt, mk, tail))
    ph = phases(blocks, loops, tanh_steps=(mk == 2))
    return {k: {c: round(v.get(c, 0)) for c in CLASSES}
            | {"total": round(sum(v.get(c, 0) for c in CLASSES)),
               "steps_per_pass": int(v["steps_per_pass"])}
            for k, v in ph.items()}


def _rows(res: dict):
    rows = ["| phase | " + " | ".join(CLASSES) + " | total | steps per loop pass |",
            "|---|" + "---|" * (len(CLASSES) + 2)]
    for k, v in res.items():
        rows.append(f"| {k} | " + " | ".join(str(v[c]) for c in CLASSES) +
                    f" | {v['total']} | {v['steps_per_pass']} |")
    return rows


def markdown(kernels: dict, cmd: str, digest: str) -> str:
    """kernels: name -> (npl, lpt, mk, counts)."""
    body = []
    for name, (npl, lpt, mk, res) in kernels.items():
        body += [f"{name}: `k_solve_gd` FP64 {npl}x{lpt}", "", *_rows(res), ""]
    rec = {"source_digest": digest,
           "kernels": {name: {"npl": npl, "lpt": lpt, "mk": mk, "phases": res}
                       for name, (npl, lpt, mk, res) in kernels.items()}}
    return "\n".join([
        "# Instructions per step of each phase of the adjoint descent kernels",
        "",
        "Static counts from the gfx950 assembly of the library's own build (wave instructions per RK4",
        "step of each phase's loop body, skippable blocks included; a body the compiler unrolled over",
        "k steps is divided by k): the plain descent, the descent with a tail hand-off and the",
        "hand-off's continuation.  Command (repository root):",
        "",
        f"    {cmd}",
        "",
        *body,
        "Machine-readable copy:",
        "",
        "```json",
        json.dumps(rec, indent=1),
        "```",
        ""])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--source", default="hj_inst_f64_1.hip")
    ap.add_argument("--npl", type=int, default=10)
    ap.add_argument("--lpt", type=int, default=1)
    ap.add_argument("--mk", type=int, default=2)
    ap.add_argument("--tail-source", default="hj_inst_r64_1.hip")
    ap.add_argument("--tail-npl", type=int, default=5)
    ap.add_argument("--tail-lpt", type=int, default=2)
    ap.add_argument("--markdown")
    args = ap.parse_args()
    kernels = {"descent": (args.npl, args.lpt, args.mk,
                           count(args.source, args.npl, args.lpt, args.mk))}
    if args.tail_lpt > 0:
        kernels["handoff"] = (args.npl, args.lpt, args.mk,
                              count(args.source, args.npl, args.lpt, args.mk, 1))
        kernels["tail"] = (args.tail_npl, args.tail_lpt, args.mk,
                           count(args.tail_source, args.tail_npl, args.tail_lpt, args.mk, 2))
    print(json.dumps({k: v[3] for k, v in kernels.items()}, indent=1))
    if args.markdown:
        import bench
        cmd = (f"python -m paper_1704_02524_amd.isa_phases --source {args.source} "
               f"--npl {args.npl} --lpt {args.lpt} --mk {args.mk} --tail-source "
               f"{args.tail_source} --tail-npl {args.tail_npl} --tail-lpt {args.tail_lpt} "
               f"--markdown {args.markdown}")
        with open(args.markdown, "w") as fh:
            fh.write(markdown(kernels, cmd, bench.source_digest()))


if __name__ == "__main__":
    main()
