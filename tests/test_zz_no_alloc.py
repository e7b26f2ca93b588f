"""ffrt_forward_static, the forward that allocates nothing (its buffers live in the library's static device
array), through the C ABI against ffrt_forward with a caller workspace: the same images bit for bit and the
same counters, on consecutive calls whose second input is smaller; and the size limit."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2302_12031_amd import ffrt
from paper_2302_12031_amd import workloads as W

pytestmark = pytest.mark.gpu

FFRT_E_OOM = 5
COUNTERS = [f for f in ffrt.STATS_FIELDS if f != "flux_on_screen"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _static_forward(handle, Pz, n_img, n_designs):
    """ffrt_forward_static on a plan handle that has no workspace."""
    irr = torch.full((n_img,), -1.0, dtype=torch.float32, device=Pz.device)
    st = torch.zeros(n_designs * ffrt.STATS_BYTES, dtype=torch.uint8, device=Pz.device)
    rc = ffrt.lib().ffrt_forward_static(handle, ctypes.c_void_p(Pz.data_ptr()), ctypes.c_void_p(irr.data_ptr()),
                                        ctypes.c_void_p(st.data_ptr()),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    ffrt._check(rc, "ffrt_forward_static")
    return irr, st


def _case(wl):
    ref = ffrt.Plan(wl.problems)
    Pz = ref.pack_cp(wl.Pz)
    st_ref = ref.new_stats()
    irr_ref = ref.forward(Pz, stats=st_ref)
    handle = ffrt.create_plan_handle(wl.problems)          # host-only plan: no workspace set
    return ref, Pz, irr_ref, st_ref, handle


def _check_same(ref, irr_ref, st_ref, irr, st, what):
    torch.cuda.synchronize()
    assert torch.equal(irr, irr_ref), f"{what}: images differ, max {float((irr - irr_ref).abs().max())}"
    a, b = ref.decode_stats(st), ref.decode_stats(st_ref)
    for f in COUNTERS:
        assert (a[f] == b[f]).all(), (what, f, a[f], b[f])
    # the flux counter is a float sum of per-workgroup partials, added in arrival order
    np.testing.assert_allclose(a["flux_on_screen"], b["flux_on_screen"], rtol=1e-6)


def test_static_forward_matches_the_workspace_forward_on_consecutive_calls():
    big = W.Workload("collimated + point", W.c1().problems + W.c3(256).problems, W.c1().Pz + W.c3(256).Pz,
                     W.c1().targets + W.c3(256).targets)
    p_small = W.collimated_problem(64, 8, 32, jitter=1, seed=5)
    small = W.Workload("small", [p_small], [W.random_heights(8, 8, 5)], [W.target_mixture(p_small, 5, 3, 3)])
    ref_b, Pz_b, irr_b, st_b, h_b = _case(big)
    ref_s, Pz_s, irr_s, st_s, h_s = _case(small)
    _say(f"[no-alloc] static forward, {big.name}: {big.num_rays} rays, {ref_b.total_img} pixels")
    irr, st = _static_forward(h_b, Pz_b, ref_b.total_img, ref_b.n_designs)
    _check_same(ref_b, irr_b, st_b, irr, st, "first call (two designs)")
    _say(f"[no-alloc] static forward, {small.name}: {small.num_rays} rays, {ref_s.total_img} pixels")
    irr, st = _static_forward(h_s, Pz_s, ref_s.total_img, ref_s.n_designs)
    _check_same(ref_s, irr_s, st_s, irr, st, "second, smaller call")
    _say("[no-alloc] static forward, first plan again")
    irr, st = _static_forward(h_b, Pz_b, ref_b.total_img, ref_b.n_designs)
    _check_same(ref_b, irr_b, st_b, irr, st, "third call (the first plan again)")
    for h in (h_b, h_s):
        ffrt.lib().ffrt_plan_destroy(h)


def test_static_forward_rejects_a_plan_larger_than_the_array():
    """70 designs of 256 x 256 pixels need more than the 32 MiB array: FFRT_E_OOM before any GPU work."""
    p = W.point_problem(64, 32, 256)
    handle = ffrt.create_plan_handle([p] * 70)
    Pz = torch.zeros(70 * 32 * 32, dtype=torch.float32, device="cuda")
    irr = torch.zeros(70 * 256 * 256, dtype=torch.float32, device="cuda")
    rc = ffrt.lib().ffrt_forward_static(handle, ctypes.c_void_p(Pz.data_ptr()), ctypes.c_void_p(irr.data_ptr()),
                                        None, None)
    assert rc == FFRT_E_OOM
    assert b"scratch" in ffrt.lib().ffrt_last_error()
    assert float(irr.abs().max()) == 0.0
    ffrt.lib().ffrt_plan_destroy(handle)
