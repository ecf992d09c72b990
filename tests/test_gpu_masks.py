"""The per-tile masks of non-zero passive scalars are an optimisation with identical
results: the stage kernel loads and transports only the scalars that can be non-zero
on a tile's stencil and skips the RK loads of planes that are zero on the whole tile.
Runs with the masks and without (cp_set_tile_masks) must agree bit for bit on states
where the masks decide something:

* the production jet 2048 x 512 with seeded droplets and crystals on 5 % of its cells
  (lognormal, realisable) and a stirred radial velocity, so that most tiles hold some
  scalars and many none, and the scalars move between tiles;
* the source-active jet on the same mesh, where the source kernels create droplets,
  activated soot and crystals in tiles whose masks were clear (the masks are widened
  by the source kernels);
* both precisions, one and two liquid populations, the autotuned tile.
"""
import numpy as np
import pytest

from paper_2504_20742_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_20742_amd import binding
    binding.load()
    return binding


def _seeded(B, m, c, prec, bimodal, seed):
    """Initial state of the case with particle fields and a stirred radial velocity."""
    s = B.Solver(m, c, prec)
    if bimodal:
        s.set_bimodal(True)
    U = s.init()
    Uh = U.double().cpu().numpy()
    het, hom, ice = inputs.particle_fields(m["nr"], m["nx"], seed=seed)
    Uh[5:9] += het
    Uh[9:13] += ice
    if bimodal:
        Uh[15:19] += hom
    Uh[2] += Uh[0] * inputs.velocity_noise(m["nr"], m["nx"], seed=seed + 1)
    s.close()
    return torch.from_numpy(Uh).to(U.dtype).cuda()


def _run(B, m, c, prec, U0, steps, masks, bimodal=False):
    s = B.Solver(m, c, prec)
    if bimodal:
        s.set_bimodal(True)
    s.set_tile_masks(masks)
    U = U0.clone()
    t = s.step_n(U, steps)
    d = s.diag(U)
    s.close()
    return U, t, d


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_masks_bit_identical_with_seeded_particles(B, prec):
    p = B.CP_FP64 if prec == "fp64" else B.CP_MIXED
    m, c = inputs.config2(0)
    U0 = _seeded(B, m, c, p, False, seed=61)
    print("masks: production jet with seeded particles, %s, 20 steps" % prec, flush=True)
    Ua, ta, da = _run(B, m, c, p, U0, 20, True)
    Ub, tb, db = _run(B, m, c, p, U0, 20, False)
    assert torch.isfinite(Ua).all()
    assert ta == tb
    assert torch.equal(Ua, Ub)
    # the particles moved: the scalar planes changed and stayed non-zero where seeded
    assert not torch.equal(Ua[5:13], U0[5:13])
    print("active cells %d, bit-identical" % da["active_cells"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_masks_bit_identical_source_active(B, prec):
    """The source creates particles in tiles whose masks were clear."""
    p = B.CP_FP64 if prec == "fp64" else B.CP_MIXED
    m, c = inputs.sa2(0)
    s = B.Solver(m, c, p)
    U0 = s.init()
    s.close()
    print("masks: source-active jet, %s, 60 steps" % prec, flush=True)
    Ua, ta, da = _run(B, m, c, p, U0, 60, True)
    Ub, tb, db = _run(B, m, c, p, U0, 60, False)
    assert da["active_cells"] > 1000 and float(Ua[5].max()) > 0.0   # droplets were made
    assert ta == tb
    assert torch.equal(Ua, Ub)


def test_masks_bit_identical_two_populations(B):
    m, c = inputs.config2(0)
    U0 = _seeded(B, m, c, B.CP_MIXED, True, seed=71)
    print("masks: two liquid populations, mixed, 20 steps", flush=True)
    Ua, ta, _ = _run(B, m, c, B.CP_MIXED, U0, 20, True, bimodal=True)
    Ub, tb, _ = _run(B, m, c, B.CP_MIXED, U0, 20, False, bimodal=True)
    assert ta == tb
    assert torch.equal(Ua, Ub)
    assert float(Ua[15].abs().max()) > 0.0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_masks_stage_buffers_written_without_masks(B, prec):
    """A stage does not store a zero scalar where its output buffer's tile mask says the
    tile already holds zero.  The two stage buffers outlive a call: here they are filled
    with particles everywhere by a run with the masks off (their masks untouched) and by
    a run under another tile shape; then a state whose particles fill only the left half
    of the mesh is stepped with the masks on.  Tiles right of that edge become
    candidates as the particles move, and read their own cells and halos: a value left
    over in a stage buffer would show in the result."""
    p = B.CP_FP64 if prec == "fp64" else B.CP_MIXED
    m, c = inputs.config2(0)
    UA = _seeded(B, m, c, p, False, seed=81)
    UB = _seeded(B, m, c, p, False, seed=82)
    UB[5:13, :, m["nx"] // 2:] = 0
    ref, tref, _ = _run(B, m, c, p, UB, 6, False)
    print("masks: stage buffers reused across mask toggles and tile shapes, %s" % prec, flush=True)
    s = B.Solver(m, c, p)
    s.set_tile(32, 8)
    U = UB.clone()
    s.step_n(U, 2)                 # masks on: the stage buffers' masks cover the left half
    s.set_tile_masks(False)
    W = UA.clone()
    s.step_n(W, 2)                 # particles everywhere in both stage buffers, masks untouched
    s.set_tile_masks(True)
    U = UB.clone()
    t = s.step_n(U, 6)
    assert t == tref
    assert torch.equal(U, ref)
    # the same after a run under another tile shape (masks of 16 x 16 tiles)
    s.set_tile(16, 16)
    W = UA.clone()
    s.step_n(W, 2)
    s.set_tile(32, 8)
    U = UB.clone()
    t = s.step_n(U, 6)
    s.close()
    assert t == tref
    assert torch.equal(U, ref)
    # the particles crossed into tiles whose masks were clear at the start
    assert float(ref[5:13, :, m["nx"] // 2:].abs().max()) > 0.0
