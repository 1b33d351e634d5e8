"""Budgeted LoD selection on the GPU (the K largest alpha'' per view, lower index first among
equal values): the whole forward path and the per-view counts equal the oracle's bit for bit,
alone and mixed with threshold views in one batch."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_09997_amd import synth
from paper_2510_09997_amd.render import Batch, Scene

from helpers import compare_forward, gpu_forward, params_struct

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


def with_budget(view, k):
    return dataclasses.replace(view, budget=int(k))


def duplicate(sc, pairs):
    for dst, src in pairs:
        for key in ("mean", "log_scale", "quat", "sh"):
            sc[key][..., dst] = sc[key][..., src]
        sc["opacity"][dst] = sc["opacity"][src]
        sc["decay"][dst] = sc["decay"][src]
    return sc


def test_budget_forward_bitexact_mixed_with_threshold_views():
    log("case: budget forward, mixed batch")
    sc = duplicate(synth.make_scene(20000, 3, "mixture", seed=31), [(11, 3), (12, 3), (500, 77)])
    base = [synth.look_at((2.0, 1.0, -9.0), width=333, height=211, s_v=2.0),
            synth.look_at((-3.0, 2.0, -8.0), width=250, height=170, s_v=1.0),
            synth.look_at((1.0, -4.0, -7.0), width=190, height=260, s_v=4.0)]
    views = [base[0], with_budget(base[1], 1500), with_budget(base[2], 6000)]
    g = gpu_forward(sc, views)
    compare_forward(g, sc, views)
    assert g["counts"][1][1] == 1500 and g["counts"][2][1] == 6000


def test_budget_cut_through_equal_alpha_keeps_lower_index():
    log("case: budget ties")
    sc = synth.make_scene(3000, 1, "uniform", seed=32)
    sc["decay"][7], sc["opacity"][7] = 1.0, 0.5          # a clearly non-zero alpha''
    sc = duplicate(sc, [(40, 7), (41, 7), (2999, 7)])
    view = synth.look_at((0.1, 0.2, -3.0), width=128, height=96, s_v=1.5)
    a2 = O.view_pass(sc, view)["rec"][:, 6].astype(np.float64)
    assert a2[7] > 0 and np.sum(a2 == a2[7]) == 4
    n = sc["n"]
    rank7 = int(np.sum(a2 > a2[7]))          # Gaussians 7, 40, 41, 2999 share alpha''
    for k in (rank7 + 1, rank7 + 2, rank7 + 3, rank7 + 4):
        v = with_budget(view, k)
        g = gpu_forward(sc, [v])
        compare_forward(g, sc, [v])
        kept = (g["flags"][:n] & 2) > 0
        want = [7, 40, 41, 2999][: k - rank7]
        assert all(kept[j] for j in want) and not any(kept[j] for j in [7, 40, 41, 2999][k - rank7:]), k


def test_budget_counts_sixty_four_views_match_oracle_and_nest():
    log("case: budget counts")
    sc = synth.make_scene(200000, 3, "mixture", seed=33)
    n = sc["n"]
    ks = np.unique(np.geomspace(1, n + 10, 64).astype(np.int64))
    pose = synth.look_at((0.0, 0.0, -6.0), width=1920, height=1080, s_v=2.0)
    views = [with_budget(pose, int(k)) for k in ks]
    scene = Scene(sc)
    b = Batch(n, views, params_struct(None))
    cnt = b.lod_count(scene).cpu().numpy()
    assert np.array_equal(cnt[:, 1], np.minimum(ks, n))
    assert np.all(np.diff(cnt[:, 2]) >= 0)
    for j in range(0, len(views), 7):
        vp = O.view_pass(sc, views[j])
        assert np.array_equal(cnt[j], vp["counts"]), (j, cnt[j], vp["counts"])
