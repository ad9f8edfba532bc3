"""nvr_march_noalloc (the allocation-free variant of nvr_march) against nvr_march,
called through the C ABI: two calls in a row on the same device, the second
with fewer rays, so the fixed scratch array holds the first call's block sums
when the second starts."""
import ctypes as C

import numpy as np
import pytest

import synth
from helpers import dev, host

pytestmark = pytest.mark.gpu


def _march_pair(md, o, d, occ, ray_begin, ray_end):
    import torch
    from paper_2304_03184_amd import _lib as L, ops as O
    n_rays = o.shape[0]
    cap = n_rays * md.max_steps
    outs = []
    for name in ("nvr_march", "nvr_march_noalloc"):
        off = torch.full((n_rays + 1,), -7, dtype=torch.int32, device="cuda")
        ray_id = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
        t = torch.full((cap,), -7.0, dtype=torch.float32, device="cuda")
        dt = torch.full((cap,), -7.0, dtype=torch.float32, device="cuda")
        x = torch.full((cap, 3), -7.0, dtype=torch.float32, device="cuda")
        n_dev = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        args = [C.byref(md), n_rays, ray_begin, ray_end, O._p(o), O._p(d), O._p(occ), cap,
                O._p(off), O._p(ray_id), O._p(t), O._p(dt), O._p(x), O._p(n_dev)]
        if name == "nvr_march":
            ws = torch.empty(max(L.lib().nvr_march_workspace(n_rays), 4), dtype=torch.uint8,
                             device="cuda")
            args.append(O._p(ws))
        args.append(O._stream())
        L.call(name, *args)
        torch.cuda.synchronize()
        n = int(n_dev.item())
        outs.append(dict(n=n, off=host(off), ray_id=host(ray_id)[:n], t=host(t)[:n],
                         dt=host(dt)[:n], x=host(x)[:n]))
    return outs


def test_march_noalloc_matches_march_on_two_calls():
    from paper_2304_03184_amd import ops as O
    w = synth.config(2)
    f = w.fields[0]
    rng = synth.rng_for(w.seed + 11)
    o, d = synth.sphere_rays(70_000, rng)          # 274 blocks of 256 rays, ragged tail
    _, occ = synth.noise_occupancy(f.occ_res, rng)
    md = O.march_desc_of(w, f)
    occ_d = dev(occ.view(np.int32))
    sizes = [(70_000, 0, 70_000), (1_000, 100, 900)]   # the second call is smaller
    for n_rays, b, e in sizes:
        print(f"march_noalloc: {n_rays} rays, range [{b}, {e})", flush=True)
        ref, got = _march_pair(md, dev(o[:n_rays]), dev(d[:n_rays]), occ_d, b, e)
        assert ref["n"] == got["n"] and ref["n"] > 0
        for k in ("off", "ray_id", "t", "dt", "x"):
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)


def test_march_noalloc_rejects_too_many_rays():
    from paper_2304_03184_amd import _lib as L, ops as O
    w = synth.config(2)
    md = O.march_desc_of(w, w.fields[0])
    n_rays = (1 << 24) + 1
    rc = L.lib().nvr_march_noalloc(C.byref(md), n_rays, 0, n_rays, None, None, None, 0, None,
                                   None, None, None, None, None, None)
    assert rc == L.NVR_EINVAL
    assert b"2^24" in L.lib().nvr_last_error()
