"""The handle's device memory from the caller's allocator (tefmm_set_allocator): PyTorch's
caching allocator serves every buffer, the results equal those of the library's own
hipMalloc bit for bit, everything is given back at destroy, and a failing allocator is
reported as TEFMM_ERR_OOM."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

K3 = (0.8, 1.5, 2.0)
D3 = (0.0, -1.2)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_torch_allocator_same_result(precision):
    import torch
    from paper_1902_05875_amd import api, inputs
    xyz, q = inputs.workload("c2", n=20_000)
    qt = torch.from_numpy(q).cuda()
    ref_h = api.TEFMM(K3, D3, p=8, precision=precision)
    ref_h.set_particles(xyz)
    ref = ref_h.evaluate(qt).cpu().numpy()
    ref_h.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    f = api.TEFMM(K3, D3, p=8, precision=precision, allocator="torch")
    tables = torch.cuda.memory_allocated() - base
    f.set_particles(xyz)
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - base
    out = f.evaluate(qt)
    torch.cuda.synchronize()
    held_eval = torch.cuda.memory_allocated() - base - out.numel() * out.element_size()
    got = out.cpu().numpy()
    print(f"{precision}: torch allocator holds {tables} B (index tables), {held / 2**20:.1f} MiB after set-up, "
          f"{held_eval / 2**20:.1f} MiB after evaluate")
    assert tables > 0 and held > tables and held_eval >= held
    assert np.array_equal(got, ref)
    f.close()
    del out
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_allocator_switch_and_autotune():
    """Switching allocators drops the geometry; set-up, autotuning (rebuilds) and evaluation
    then run on torch's memory."""
    import torch
    from paper_1902_05875_amd import api, inputs
    xyz, q = inputs.workload("c2", n=20_000)
    qt = torch.from_numpy(q).cuda()
    f = api.TEFMM(K3, D3, p=6, precision="fp32")
    f.set_particles(xyz)
    a = f.evaluate(qt).cpu().numpy()
    f.set_allocator("torch")
    with pytest.raises(api.TefmmError):
        f.evaluate(qt)  # no geometry any more
    f.set_particles(xyz)
    f.autotune()
    b = f.evaluate(qt).cpu().numpy()
    assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(a)
    f.set_allocator(None)
    f.set_particles(xyz)
    c = f.evaluate(qt).cpu().numpy()
    assert np.linalg.norm(a - c) <= 1e-4 * np.linalg.norm(a)
    f.close()


def test_failing_allocator_reports_oom():
    from paper_1902_05875_amd import api
    calls = []

    def alloc(nbytes, user):
        calls.append(nbytes)
        return None

    def free(ptr, user):
        raise AssertionError("nothing was allocated")

    fa, ff = api.ALLOC_FN(alloc), api.FREE_FN(free)
    f = api.TEFMM(K3, D3, p=6)
    rc = api.lib().tefmm_set_allocator(f.h, fa, ff, None)
    assert rc == -6 and calls, rc  # TEFMM_ERR_OOM on the first request
    assert "out of memory" in api.lib().tefmm_last_error(f.h).decode().lower()
    api.lib().tefmm_set_allocator(f.h, api.ALLOC_FN(), api.FREE_FN(), None)
    f.close()
