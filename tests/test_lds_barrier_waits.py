"""Generated-code check: no workgroup barrier is reached with an LDS operation still in flight.

Every kernel source is compiled for gfx950 to assembly (device code only) and each kernel's control
flow is followed: a barrier (s_barrier) that some path reaches after an LDS instruction (ds_*) with
no s_waitcnt lgkmcnt(0) in between lets another wave read an LDS slot before the store to it has
landed.  The compiler can leave out that wait where the stores come from a loop's previous
iteration; the kernels that need it drain the counter themselves before the barrier.
"""
import os
import re
import shutil
import subprocess
from collections import defaultdict

import pytest

from paper_2406_06283_amd import build as B

HIP_SOURCES = [s for s in B.SOURCES if s.endswith(".hip")]


def _kernels(text):
    cur, body = None, []
    for ln in text.splitlines():
        m = re.match(r"^(_Z\S+):\s", ln)
        if m and "@" in ln:
            cur, body = m.group(1), []
            continue
        if cur is None:
            continue
        if ln.startswith(".Lfunc_end"):
            yield cur, body
            cur = None
        else:
            body.append(ln)


def _unsafe_barriers(body):
    """Blocks holding a barrier that a path reaches with an LDS operation not yet waited for."""
    order, blocks = ["entry"], defaultdict(list)
    for ln in body:
        m = re.match(r"^(\.LBB\S+):", ln) or re.match(r"^; (%bb\.\S+):", ln)
        if m:
            order.append(m.group(1))
            continue
        s = ln.strip()
        if s and not s.startswith((";", ".")):
            blocks[order[-1]].append(s)
    succ = defaultdict(list)
    for i, b in enumerate(order):
        last = blocks[b][-1] if blocks[b] else ""
        target = re.findall(r"(\.LBB\S+)", last)
        if last.startswith("s_branch"):
            succ[b] += target[:1]
            continue
        if last.startswith("s_endpgm"):
            continue
        if last.startswith("s_cbranch"):
            succ[b] += target[:1]
        if i + 1 < len(order):
            succ[b].append(order[i + 1])

    def run(b, pending, hits=None):
        for s in blocks[b]:
            op = s.split()[0]
            if op.startswith("ds_"):
                pending = True
            elif op == "s_waitcnt" and "lgkmcnt(0)" in s:
                pending = False
            elif op == "s_barrier" and pending and hits is not None:
                hits.append(b)
        return pending

    entry = {b: False for b in order}
    changed = True
    while changed:
        changed = False
        for b in order:
            if run(b, entry[b]):
                for t in succ[b]:
                    if not entry.get(t, True):
                        entry[t] = changed = True
    hits = []
    for b in order:
        run(b, entry[b], hits)
    return hits


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_no_barrier_reached_with_lds_operations_in_flight(tmp_path):
    procs = []
    for src in HIP_SOURCES:
        out = tmp_path / (src + ".s")
        cmd = [B.hipcc(), *[f for f in B.HIP_FLAGS if not f.startswith("-W")], "-x", "hip", "-S", "--cuda-device-only",
               os.path.join(B.CSRC, src), "-o", str(out)]
        procs.append((src, out, subprocess.Popen(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE)))
    bad, nbarriers = [], 0
    for src, out, p in procs:
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, err.decode(errors="replace")[-2000:]
        text = out.read_text()
        nbarriers += text.count("s_barrier")
        for name, body in _kernels(text):
            hits = _unsafe_barriers(body)
            if hits:
                bad.append((src, name, hits[:4]))
    assert nbarriers > 50            # the scan saw the kernels' barriers
    assert not bad, bad
