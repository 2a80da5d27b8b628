"""The autotuner's on-disk cache (MXP_AUTOTUNE_CACHE): a tuned choice is
written under its key, a later problem of the same key takes the cached
choice instead of timing candidates, and a file that is not a tile cache is
neither trusted nor overwritten."""
import json
import os

import pytest

import workloads as wl

from gpu_util import announce, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_03617_amd as mxp  # noqa: E402
from oracle import matfun, operator as op  # noqa: E402


@pytest.mark.parametrize("dims", [2, 3])
def test_tile_cache_round_trip(tmp_path, monkeypatch, dims):
    path = str(tmp_path / "tiles.json")
    monkeypatch.setenv("MXP_AUTOTUNE_CACHE", path)
    n = (97, 61) if dims == 2 else (40, 17, 27)
    prob = wl.small_problem(n, layer=6 if dims == 2 else 4, ppw=10, inhomogeneous=True, seed=9, name="cache")
    announce("tile cache", dims, n)
    ctx = mxp.Context(0)
    x = to_dev(wl.random_vector(prob.npts, 2), torch.complex64)
    y = torch.empty_like(x)
    t, s = prob.default_t(), prob.default_shift()
    # 1. the first problem tunes and writes its choice
    P = mxp.Problem(ctx, prob)
    mxp.mxp_apply_exp(P, t, s, x, y)
    tuned = mxp.mxp_get_tiles(P, mxp.MXP_PREC_MIXED)
    P.close()
    cache = json.load(open(path))
    keys = [k for k in cache if "c64" in k and f"{dims}d" in k]
    assert len(keys) == 1
    key = keys[0]
    assert cache[key][:3] == [tuned["K"], tuned["NX"], tuned["Ly"]]
    # 2. a cached choice (another valid one, with a marker time) is taken as it is
    other = [2, 1, 8, 1.25] if dims == 2 else ([1, 1, 0, 1.25] if tuned["K"] == 2 else [2, 1, 16, 1.25])
    cache[key] = other
    json.dump(cache, open(path, "w"))
    P = mxp.Problem(ctx, prob)
    mxp.mxp_apply_exp(P, t, s, x, y)
    got = mxp.mxp_get_tiles(P, mxp.MXP_PREC_MIXED)
    assert [got["K"], got["NX"], got["Ly"]] == other[:3] and got["us_per_level"] == 1.25
    ref = matfun.exp_action(op.helmholtz(prob, s), t, to_host(x).astype("complex128"))
    assert rel(to_host(y), ref) <= 1e-5  # the cached shape computes the same action
    P.close()
    # 3. an entry this build cannot run is ignored (the candidates are timed)
    cache[key] = [9, 3, 0, 1.25]
    json.dump(cache, open(path, "w"))
    P = mxp.Problem(ctx, prob)
    mxp.mxp_apply_exp(P, t, s, x, y)
    assert mxp.mxp_get_tiles(P, mxp.MXP_PREC_MIXED)["us_per_level"] != 1.25
    P.close()
    # 4. a file that is not a tile cache is neither used nor overwritten
    with open(path, "w") as fh:
        fh.write("not a cache\n")
    P = mxp.Problem(ctx, prob)
    mxp.mxp_apply_exp(P, t, s, x, y)
    assert mxp.mxp_get_tiles(P, mxp.MXP_PREC_MIXED)["us_per_level"] != 1.25
    assert open(path).read() == "not a cache\n"
    P.close()
    ctx.close()
    assert not os.path.exists(path + ".tmp")
