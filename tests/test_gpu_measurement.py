"""GPU checks of the two measurement aids the benchmark relies on:
dwf_stream_copy, whose known byte count calibrates the memory counters,
copies exactly what it is given and nothing past it; dwf_time_kernels
reports for every inner kernel the algorithmic bytes of the per-site model
(every operand read or written once) that the roofline divides by.
"""
import numpy as np
import pytest

from _util import Problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nontemporal", [False, True], ids=["cached", "nontemporal"])
@pytest.mark.parametrize("nbytes", [16, 48, 1 << 20, (64 << 20) + 16 * 37])
def test_stream_copy_is_exact(nontemporal, nbytes):
    import torch

    import paper_1101_0423_amd as dwf
    print(f"[copy] {nbytes} bytes nontemporal={nontemporal}", flush=True)
    torch.manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
    out = torch.full((nbytes + 256,), 0xA5, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    # the library never uses the legacy null stream, torch's default one
    with pytest.raises(ValueError):
        dwf.stream_copy(src, out[:nbytes], nontemporal=nontemporal)
    side = torch.cuda.Stream()
    dwf.stream_copy(src, out[:nbytes], nontemporal=nontemporal, stream=side.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(out[:nbytes], src)
    assert bool((out[nbytes:] == 0xA5).all())


def test_time_kernels_reports_the_bytes_model():
    import paper_1101_0423_amd as dwf
    P = Problem.workload("shamir_4x4x4x4_ns8")
    c = P.context()
    try:
        p = dwf.default_params(inner_prec=dwf.PREC_FP32)
        # no workspace before the first solve with these parameters
        with pytest.raises(dwf.DwfError) as ei:
            c.time_kernels(params=p, launches=2)
        assert ei.value.code == dwf.DWF_EINVAL
        x, st, rc = c.solve(P.b, params=p)
        assert rc == dwf.DWF_OK
        ms, by = c.time_kernels(params=p, launches=3)
    finally:
        c.close()
    v4h = int(np.prod(P.dims)) // 2
    v5h = v4h * P.ns
    sb = yb = 96.0 * v5h            # FP32 spinor / FP32 solution vector
    lb = 8.0 * 48.0 * v4h           # 8 links of 12 FP32 reals per 4D site
    model = dict(T=2 * sb, A=2 * sb + lb, B=4 * sb + lb, C=2 * sb + lb, D=5 * sb + 2 * yb + lb)
    print(f"[time] ms {ms}", flush=True)
    for k in "TABCD":
        assert by[k] == model[k], (k, by[k], model[k])
        assert ms[k] > 0
