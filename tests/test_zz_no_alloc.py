"""The mixed-batch entry point that allocates no device memory
(ksym_mixed_run_noalloc) against the plan path (ksym_plan_create +
ksym_plan_run) on the same groups and options, through the C ABI: bitwise
equal outputs and counters, on two calls in a row with the second batch
smaller than the first (the fixed tables keep the first call's contents), in
float32 at the tuned mixed-batch shape and in float64."""

import numpy as np
import pytest

import synth
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ksym():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_6291_amd as k
    return k


def _outputs(k, s, dtype):
    nl, nd, nphi = (3, 9, (3, s)) if k == 3 else (2, 4, (s,))
    return {"lam": torch.full((nl, s), -7.0, dtype=dtype, device="cuda"),
            "D": torch.full((nd, s), -7.0, dtype=dtype, device="cuda"),
            "phi": torch.full(nphi, -7.0, dtype=dtype, device="cuda"),
            "flags": torch.full((s,), 255, dtype=torch.uint8, device="cuda")}


def _case(total, ngroups, seed, dtype):
    """Groups of 2x2 and 3x3 matrices (log-uniform sizes, one empty group, one
    of a single matrix); every third 3x3 group follows the precision recipe
    (near-degenerate and repeated spectra, so that matrices are refined), the
    others have N(0, 1) entries.  Two output sets for the same inputs."""
    sizes, kinds = synth.mixed_group_sizes(total, ngroups, lo=100, hi=2e4, seed=seed)
    sizes[1] = 0
    sizes[2] = 1
    rng = np.random.default_rng(seed)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    a, b = [], []
    for g, (s, k) in enumerate(zip(sizes, kinds)):
        s, k = int(s), int(k)
        if k == 3 and g % 3 == 0 and s > 0:
            P = synth.make_precision(s, seed=seed + g, dtype=npdt)
        else:
            P = rng.standard_normal((6 if k == 3 else 3, s)).astype(npdt)
        t = to_dev(P, dtype)
        a.append((k, t, _outputs(k, s, dtype)))
        b.append((k, t, _outputs(k, s, dtype)))
    return a, b


def _same(a, b, tag):
    for g, ((k, _, oa), (_, _, ob)) in enumerate(zip(a, b)):
        for key in oa:
            assert torch.equal(oa[key], ob[key]), (tag, g, k, key)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_noalloc_matches_plan_on_two_calls(ksym, dtype):
    tdt = torch.float32 if dtype == "float32" else torch.float64
    dt = ksym.F32 if dtype == "float32" else ksym.F64
    opts = ksym.tuned_opts("mixed", dt) if dtype == "float32" else None
    ws = ksym.workspace()
    refined = []
    for call, (total, ngroups, seed) in enumerate(((400000, 120, 311), (30000, 17, 312))):
        print(f"[noalloc] {dtype} call {call}: {ngroups} groups, {total} matrices", flush=True)
        ga, gb = _case(total, ngroups, seed, tdt)
        plan = ksym.Plan(ga, opts=opts)
        plan.run()
        ksym.mixed_run_noalloc(gb, opts=opts, ws=ws)
        torch.cuda.synchronize()
        _same(ga, gb, (dtype, call))
        assert torch.equal(plan.ws[:2], ws[:2]), (plan.ws[:2], ws[:2])
        refined.append(int(ws[0].item()))
        # every matrix written (no sentinel left in a non-empty group)
        for k, t, o in gb:
            if t.shape[1]:
                assert not torch.any(o["flags"] == 255)
        plan.close()
    assert refined[0] > 0, refined
