"""Static check of the compiled kernels: every loop that contains a barrier
must be controlled by scalar (wave-uniform) branches.

A loop whose exit the compiler sees as per-lane is lowered with exec-mask
branches.  If a single-lane region (``if (tid == 0)``) is then threaded across
the back-edge, lanes of one wave can reach the loop's barriers on different
passes, and the workgroup deadlocks.  This module builds the control-flow
graph of each kernel from the AMDGCN assembly that hipcc emits (``-S``), finds
natural loops through dominators, and reports barrier loops whose back-edge
or exits test the exec mask.

Usage: ``python -m paper_1312_0138_amd.check_barriers`` (exit status 1 when a
divergent barrier loop is found).
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile

from .build import FLAGS, HIPCC, SRC


def device_asm(out_path: str, src: str = SRC) -> str:
    """Compile the library's device code to AMDGCN assembly at out_path."""
    flags = [f for f in FLAGS if f not in ("-shared", "-fPIC")]
    subprocess.run([HIPCC, *flags, "--cuda-device-only", "-S", "-o", out_path, src], check=True,
                   capture_output=True)
    return out_path


def _kernels(lines):
    kernels, cur = [], None
    for ln in lines:
        m = re.match(r"^(_Z\S+):", ln)
        if m:
            cur = {"name": m.group(1), "blocks": [["entry", []]]}
            kernels.append(cur)
            continue
        if cur is None:
            continue
        if re.match(r"^\s*\.Lfunc_end", ln):
            cur = None
            continue
        m = re.match(r"^(\.LBB\w+):", ln) or re.match(r"^; %(bb\.\d+):", ln)
        if m:
            cur["blocks"].append([m.group(1), []])
            continue
        cur["blocks"][-1][1].append(ln.strip())
    return kernels


def _barrier_loops(kernel):
    blocks = kernel["blocks"]
    names = [b[0] for b in blocks]
    idx = {n: i for i, n in enumerate(names)}
    n = len(blocks)
    succ = []
    for i, (_, ins) in enumerate(blocks):
        s, term = [], False
        for x in ins:
            m = re.match(r"(s_cbranch_\w+|s_branch)\s+(\.LBB\w+)", x)
            if m:
                s.append((idx[m.group(2)], m.group(1)))
                term = term or m.group(1) == "s_branch"
            term = term or x.startswith("s_endpgm")
        if not term and i + 1 < n:
            s.append((i + 1, "fall"))
        succ.append(s)
    pred = [[] for _ in range(n)]
    for i in range(n):
        for j, _ in succ[i]:
            pred[j].append(i)
    dom = [set(range(n)) for _ in range(n)]
    dom[0] = {0}
    changed = True
    while changed:
        changed = False
        for i in range(1, n):
            ps = [dom[p] for p in pred[i]]
            nd = ({i} | set.intersection(*ps)) if ps else {i}
            if nd != dom[i]:
                dom[i] = nd
                changed = True
    loops = []
    for b in range(n):
        for h, kind in succ[b]:
            if h not in dom[b]:
                continue  # not a back-edge
            body, stack = {h, b}, [b]
            while stack:
                x = stack.pop()
                if x == h:
                    continue
                for p in pred[x]:
                    if p not in body:
                        body.add(p)
                        stack.append(p)
            if not any("s_barrier" in x for i in body for x in blocks[i][1]):
                continue
            exits = [kd for i in body for j, kd in succ[i] if j not in body]
            divergent = "exec" in kind or any("exec" in kd for kd in exits)
            loops.append((names[h], names[b], kind, "DIVERGENT" if divergent else "uniform"))
    return loops


def check_text(asm_text: str):
    """{kernel name: [(header, latch, branch, 'DIVERGENT' | 'uniform'), ...]}."""
    return {k["name"]: _barrier_loops(k) for k in _kernels(asm_text.splitlines())}


def divergent_barrier_loops(asm_text: str):
    return {k: [l for l in v if l[3] == "DIVERGENT"] for k, v in check_text(asm_text).items()
            if any(l[3] == "DIVERGENT" for l in v)}


def main(argv=None) -> int:
    argv = sys.argv[1:] if argv is None else argv
    if argv:
        text = open(argv[0]).read()
    else:
        with tempfile.TemporaryDirectory() as d:
            text = open(device_asm(os.path.join(d, "k.s"))).read()
    bad = divergent_barrier_loops(text)
    for k, v in check_text(text).items():
        print(("BAD " if k in bad else "ok  ") + k, len(v), "barrier loop(s)", bad.get(k, ""))
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main())
