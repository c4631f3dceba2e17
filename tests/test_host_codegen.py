"""Generated-code invariant of the HIP kernels (host only: device assembly
for gfx950 produced by hipcc with the library's own flags).

Workgroups publish values through LDS and a barrier (the persistent tile
loops, the staged source and z tiles).  A barrier publishes an LDS write
only once the write has completed, so on every path from an LDS write to a
barrier the code must wait for the LDS counter to drain (lgkmcnt(0)).  The
compiler normally inserts that wait; a loop whose back-edge carried an LDS
write straight to the loop-top barrier once came out without it, letting
waves read a stale tile index.  This test checks every kernel's control-flow
graph for such a path."""
import os
import re
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("hrir_build_asm", os.path.join(ROOT, "paper_1502_03162_amd",
                                                                                  "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _functions(text):
    lines = text.split("\n")
    i = 0
    while i < len(lines):
        m = re.match(r"^(\w+):\s*;\s*@", lines[i])
        if m:
            j = i + 1
            while j < len(lines) and not lines[j].startswith(".Lfunc_end"):
                j += 1
            yield m.group(1), lines[i + 1:j]
            i = j
        i += 1


def _blocks(lines):
    """Basic blocks: a label starts one, a branch or s_endpgm ends one (the
    next instruction then starts an unlabelled block)."""
    out, cur, name, n_anon = [], [], "entry", 0
    for line in lines:
        m = re.match(r"^(\.LBB\w+):", line)
        if m:
            if cur or name != "entry":
                out.append((name, cur))
            name, cur = m.group(1), []
            continue
        s = line.strip()
        if not s or s.startswith((";", ".")):
            continue
        cur.append(s)
        if s.split()[0].startswith(("s_branch", "s_cbranch", "s_endpgm", "s_setpc")):
            out.append((name, cur))
            n_anon += 1
            name, cur = f"{name}+{n_anon}", []
    out.append((name, cur))
    return out


def _is_lds_write(op):
    return op.startswith("ds_") and not op.startswith(("ds_read", "ds_bpermute", "ds_permute", "ds_swizzle",
                                                         "ds_nop"))


def _drains_lds(ins):
    return ins.startswith("s_waitcnt") and ("lgkmcnt(0)" in ins or re.match(r"s_waitcnt\s+0$", ins))


def unwaited_barriers(lines):
    """Barriers reachable from an LDS write with no lgkmcnt(0) in between
    (forward may-analysis over the basic blocks of one function)."""
    bl = _blocks(lines)
    index = {n: k for k, (n, _) in enumerate(bl)}
    succ = []
    for k, (_, ins) in enumerate(bl):
        last = ins[-1].split() if ins else [""]
        if last[0] == "s_branch":
            succ.append([index[last[1]]])
        elif last[0].startswith("s_cbranch"):
            succ.append([index[last[1]]] + ([k + 1] if k + 1 < len(bl) else []))
        elif last[0] in ("s_endpgm", "s_setpc_b64"):
            succ.append([])
        else:
            succ.append([k + 1] if k + 1 < len(bl) else [])
    pending_in = [False] * len(bl)
    seen = [False] * len(bl)
    bad = set()
    work = [0]
    while work:
        k = work.pop()
        st = pending_in[k]
        for ins in bl[k][1]:
            op = ins.split()[0]
            if _is_lds_write(op):
                st = True
            elif _drains_lds(ins):
                st = False
            elif op == "s_barrier" and st:
                bad.add(bl[k][0])
        seen[k] = True
        for q in succ[k]:
            if (st and not pending_in[q]) or not seen[q]:
                pending_in[q] = pending_in[q] or st
                work.append(q)
    return sorted(bad)


def test_audit_detects_a_missing_wait():
    """The analysis itself: a back-edge LDS write reaching the loop-top
    barrier is found; the same loop with the wait is clean."""
    bad_loop = """k:  ; @k
\tv_mov_b32_e32 v1, 0
\ts_waitcnt lgkmcnt(0)
.LBB0_1:
\ts_barrier
\tds_read_b32 v2, v1
\ts_waitcnt lgkmcnt(0)
\tds_write_b32 v1, v2
\ts_cbranch_scc1 .LBB0_1
\ts_endpgm
.Lfunc_end0:
"""
    good_loop = bad_loop.replace("\tds_write_b32 v1, v2\n", "\tds_write_b32 v1, v2\n\ts_waitcnt lgkmcnt(0)\n")
    (name, lines), = list(_functions(bad_loop))
    assert unwaited_barriers(lines) == [".LBB0_1"]
    (name, lines), = list(_functions(good_loop))
    assert unwaited_barriers(lines) == []


def test_every_barrier_waits_for_lds_writes(tmp_path):
    b = _build_module()
    try:
        b.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    sources = [s for s in b.SOURCES if s.endswith(".hip")]
    with ThreadPoolExecutor(max_workers=4) as ex:
        paths = list(ex.map(lambda s: b.assemble(s, str(tmp_path / (s + ".s"))), sources))
    problems, n_kernels = [], 0
    for src, path in zip(sources, paths):
        for name, lines in _functions(open(path).read()):
            n_kernels += 1
            bad = unwaited_barriers(lines)
            if bad:
                problems.append((src, name, bad))
    assert n_kernels > 50
    assert not problems, problems
