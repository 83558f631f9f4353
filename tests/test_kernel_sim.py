"""CPU checks of the fused kernel's tile algorithm through its model
(tests/kernel_sim.py): the result equals the oracle, the barrier schedule is
free of LDS races for double and single buffering (and removing any one of
its barriers is caught), unwritten LDS never reaches a stored output, every
tile height gives the same bits, and consecutive tiles may share the
double-buffered planes without a barrier between them (the fused
multi-level tail), which single-buffered planes may not."""
import numpy as np
import pytest

import kernel_sim as ks
import oracle

ROWS = {"cdf53": (2, 3), "cdf97": (2, 3, 4), "dd137": (3, 6)}
SIZES = [(2, 2), (5, 3), (37, 22), (70, 61), (130, 33)]


def image(w, h, seed):
    return np.random.default_rng(seed).integers(0, 256, size=(h, w)).astype(np.float64)


@pytest.mark.parametrize("wav", ["cdf53", "cdf97", "dd137"])
def test_model_matches_the_oracle_and_is_race_free(wav):
    """FP64 model vs the FP64 oracle, one level, every height and both
    bufferings; the race checker raises on any unsynchronised plane access,
    and the NaN-filled planes would show in an output that read an unwritten
    cell."""
    for i, (w, h) in enumerate(SIZES):
        x = image(w, h, 700 + i)
        ref = oracle.forward(x, wav, 1)
        for rb in ROWS[wav]:
            for nb in (2, 1):
                y = ks.forward(x, wav, rb, nb)
                assert np.all(np.isfinite(y)), (wav, w, h, rb, nb)
                assert np.abs(y - ref).max() < 1e-9, (wav, w, h, rb, nb)
                z = ks.inverse(y, wav, rb, nb)
                assert np.all(np.isfinite(z)), (wav, w, h, rb, nb)
                assert np.abs(z - oracle.inverse(y, wav, 1)).max() < 1e-9, (wav, w, h, rb, nb)


BARRIERS = {2: ["predict", "update"],
            1: ["predict", "update", "before_predict_publish", "before_update_publish"]}


@pytest.mark.parametrize("nb", [2, 1])
@pytest.mark.parametrize("direction", ["forward", "inverse"])
def test_every_barrier_is_needed(direction, nb):
    """Dropping any one barrier of the schedule makes some wavefront read a
    plane row another wavefront writes in the same epoch (or overwrite one it
    reads): the checker must catch it.  9/7 (two pairs) so that every barrier
    kind occurs."""
    x = image(130, 70, 710)
    run = ks.forward if direction == "forward" else ks.inverse
    arg = x if direction == "forward" else ks.forward(x, "cdf97", 4, nb)
    run(arg, "cdf97", 4, nb)  # the full schedule passes
    for name in BARRIERS[nb]:
        with pytest.raises(ks.Race):
            run(arg, "cdf97", 4, nb, barriers={name: False})


def test_double_buffering_needs_one_barrier_per_step_only():
    """The two single-buffering barriers are exactly what double buffering
    saves: with separate planes for predict and update, the schedule without
    them is race-free."""
    x = image(70, 61, 711)
    for wav in ("cdf53", "cdf97", "dd137"):
        ks.forward(x, wav, ROWS[wav][-1], 2,
                   barriers={"before_predict_publish": False, "before_update_publish": False})


@pytest.mark.parametrize("wav", ["cdf53", "cdf97", "dd137"])
def test_heights_and_bufferings_give_identical_fp32_bits(wav):
    x = image(130, 97, 712).astype(np.float32)
    outs = [ks.forward(x, wav, rb, nb, np.float32) for rb in ROWS[wav] for nb in (2, 1)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    invs = [ks.inverse(outs[0].astype(np.float32), wav, rb, nb, np.float32)
            for rb in ROWS[wav] for nb in (2, 1)]
    for o in invs[1:]:
        assert np.array_equal(o, invs[0])


@pytest.mark.parametrize("wav", ["cdf53", "cdf97", "dd137"])
def test_consecutive_tiles_share_double_buffered_planes(wav):
    """One work-group running a level's tiles back to back on the same
    planes (no barrier between tiles) is race-free and gives the oracle's
    result, in both directions, at the tallest height (the tail's)."""
    x = image(130, 70, 720)
    rb = ROWS[wav][-1]
    y = ks.forward(x, wav, rb, 2, shared_planes=True)
    assert np.abs(y - oracle.forward(x, wav, 1)).max() < 1e-9
    z = ks.inverse(y, wav, rb, 2, shared_planes=True)
    assert np.abs(z - oracle.inverse(y, wav, 1)).max() < 1e-9


@pytest.mark.parametrize("direction", ["forward", "inverse"])
def test_single_buffered_planes_need_a_barrier_between_tiles(direction):
    """With one plane buffer, the next tile's first publication overwrites
    rows the previous tile's last step still reads in the same epoch."""
    x = image(130, 70, 721)
    arg = x if direction == "forward" else ks.forward(x, "cdf97", 4, 2)
    run = ks.forward if direction == "forward" else ks.inverse
    with pytest.raises(ks.Race):
        run(arg, "cdf97", 4, 1, shared_planes=True)
