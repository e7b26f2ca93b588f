"""The benchmark's per-ray FP32 operation counts against the FP32 instructions the hardware counted.

bench.py prices the trace kernels with a table of algorithmic FP32 operations per ray (a fixed part and a part
per Newton iteration, counted stage by stage from the kernels' formulation).  The committed rocprofv3
summaries under profiles/ hold what the GPU executed per ray (SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F32 x 64 lanes
/ rays, an FMA counted as 2).  Executed counts include lanes left idle in divergent branches and the
few rays a kernel re-traces, so the two need not be equal; the table must stay within 10 % of them, with the
forward's Newton iterations taken from the count its own statistics recorded in the same summary.
"""
import os
import re

import pytest

import bench
from paper_2302_12031_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL = 0.10


def _counted(name, kernel):
    text = open(os.path.join(ROOT, "profiles", name)).read()
    head = None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if line.startswith("| kernel"):
            head = cells
        elif head and line.startswith("|") and cells[0] == kernel:
            return float(cells[head.index("FP32 flops/ray")]), text
    raise AssertionError(f"{kernel} not in {name}")


def _per_ray(wl, kernel, iters, steps=None):
    tot, _ = bench.algorithmic_flops(wl, kernel, iters, steps)
    return tot / wl.num_rays


def test_point_source_forward_and_adjoint_match_the_counters():
    wl = W.c4()
    fwd, text = _counted("trace_kernels_c4_valu_counters.md", "ffrt::k_forward_w3<3, 3, 3, 3, 1>")
    adj, _ = _counted("trace_kernels_c4_valu_counters.md", "ffrt::k_adjoint_w3<3, 3, 3, 1>")
    iters = float(re.search(r"\(([0-9.]+) Newton iterations per ray", text).group(1))
    t_fwd = _per_ray(wl, "forward", 0.0, [iters * wl.num_rays])
    t_adj = _per_ray(wl, "adjoint", 0.0)          # the adjoint of a step reads the stored exit roots
    assert abs(t_fwd - fwd) <= TOL * fwd, (t_fwd, fwd)
    assert abs(t_adj - adj) <= TOL * adj, (t_adj, adj)


def test_collimated_forward_and_adjoint_match_the_counters():
    wl = W.c2()
    fwd, _ = _counted("trace_kernels_c2_valu_counters.md", "ffrt::k_forward<3, 3, 3, 2, 0>")
    adj, _ = _counted("trace_kernels_c2_valu_counters.md", "ffrt::k_adjoint<3, 3, 3, 0>")
    assert abs(_per_ray(wl, "forward", 0.0) - fwd) <= TOL * fwd
    assert abs(_per_ray(wl, "adjoint", 0.0) - adj) <= TOL * adj


@pytest.mark.parametrize("iters", [1.0, 2.5])
def test_search_steps_enter_linearly(iters):
    """A forward with twice the Newton iterations per ray costs newton_iter more per iteration and ray."""
    wl = W.c3(64)
    a = _per_ray(wl, "forward", iters)
    b = _per_ray(wl, "forward", 2 * iters)
    assert abs((b - a) - bench.FLOPS["point"]["newton_iter"] * iters) < 1e-9
