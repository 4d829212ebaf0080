"""The network on the matrix cores (NEP_NETWORK_MFMA): the descriptor x hidden
layer product of Eq. 2 and its transpose over a wavefront's 64 beads as FP32
MFMAs.  Parity with the FP64 oracle at the contract tolerances, agreement with
the vector-ALU network up to rounding, partial last wavefronts, every hidden
width it takes, an MD trajectory, and the models it refuses."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import compare_efv, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _replica(spec, params, system, skin, engine):
    from paper_2603_01234_amd import engine as E
    model = E.Model.from_spec(spec, params).set_network(engine)
    rep = E.Replica(model, system.pos_f32(), system.types, system.box, system.pbc, skin=skin, vel=system.vel)
    rep._model_keep = model
    return rep


def _oracle(spec, params, rep, system, targets=None):
    return oracle.efv(spec, params.astype(np.float32).astype(np.float64), rep.positions().astype(np.float64),
                      system.types, np.asarray(rep.box, np.float32).astype(np.float64), system.pbc,
                      targets=targets)


def test_mfma_network_parity_config0():
    spec, params, system, opts = W.config0()
    rep = _replica(spec, params, system, opts["skin"], "mfma")
    rep.efv()
    compare_efv(rep, _oracle(spec, params, rep, system), system.n, label="config0-mfma")


@pytest.mark.parametrize("n, hidden", [(37, 30), (200, 12), (131, 50), (64, 16)])
def test_mfma_network_partial_wavefronts_and_widths(n, hidden):
    """n not a multiple of 64 (lanes past the end take part in the matrix
    products with a dummy bead), hidden widths padded to 16, 32 and 64."""
    rng = np.random.default_rng(n + hidden)
    spec = W.water_spec(hidden)
    params = W.draw_params(spec, rng)
    system = W.water_random_sites(rng, n, 33.4)
    rep = _replica(spec, params, system, 0.0, "mfma")
    rep.efv()
    compare_efv(rep, _oracle(spec, params, rep, system), system.n, label=f"mfma-n{n}-h{hidden}")


def test_mfma_and_valu_networks_agree_config1():
    spec, params, system, opts = W.config1()
    out = {}
    for eng in ("valu", "mfma"):
        rep = _replica(spec, params, system, opts["skin"], eng)
        rep.efv()
        out[eng] = (rep.forces().astype(np.float64), rep.site_energies().astype(np.float64),
                    rep.virials().astype(np.float64))
    Fv, Uv, Wv = out["valu"]
    Fm, Um, Wm = out["mfma"]
    assert rel_rms(Fm, Fv) < 1e-6
    assert np.abs(Um - Uv).max() < 2e-7
    assert rel_rms(Wm, Wv) < 1e-6
    # and against the oracle on sampled beads
    targets = np.random.default_rng(3).choice(system.n, 150, replace=False)
    rep = _replica(spec, params, system, opts["skin"], "mfma")
    rep.efv()
    compare_efv(rep, _oracle(spec, params, rep, system, targets=targets), system.n, targets=targets,
                label="config1-mfma")


def test_mfma_network_md_config0_tracks_oracle():
    """512 beads from rest, dt = 2 fs, 100 NVE steps with the matrix-core
    network: energies per step and final positions against the FP64 oracle
    (the tolerances of the vector-ALU MD test)."""
    spec, params, system, opts = W.config0()
    rep = _replica(spec, params, system, opts["skin"], "mfma")
    rep.efv()
    n_steps = opts["steps"]
    Ep = torch.zeros(n_steps, dtype=torch.float64, device="cuda")
    Ek = torch.zeros(n_steps, dtype=torch.float64, device="cuda")
    rep.md(n_steps, opts["dt"], [W.WATER_MASS], rebuild_every=opts["rebuild_every"], E_pot=Ep, E_kin=Ek)
    Ep, Ek = Ep.cpu().numpy(), Ek.cpu().numpy()
    p32 = system.pos_f32().astype(np.float64)
    pos, vel, F, box, Epo, Eko = oracle.md(spec, params.astype(np.float32).astype(np.float64), p32,
                                           np.zeros_like(p32), system.types, [W.WATER_MASS],
                                           system.box.astype(np.float32), system.pbc, opts["dt"], n_steps)
    n = system.n
    assert np.abs(Ep - Epo).max() / n < 1e-5 and np.abs(Ek - Eko).max() / n < 1e-5
    L = system.box.astype(np.float32).astype(np.float64)
    dpos = rep.positions().astype(np.float64) - pos
    dpos -= L * np.round(dpos / L)
    assert np.abs(dpos).max() < 1e-4


def test_mfma_network_refuses_what_it_does_not_take():
    from paper_2603_01234_amd import binding as B
    from paper_2603_01234_amd import engine as E
    rng = np.random.default_rng(9)
    two = W.aacg_gold_spec(30)           # two bead types
    m2 = E.Model.from_spec(two, W.draw_params(two, rng))
    assert B.nep_model_set_network(m2.handle, B.NEP_NETWORK_MFMA) == B.NEP_ERR_UNSUPPORTED
    narrow = W.water_spec(8)             # hidden width padded to 8
    m8 = E.Model.from_spec(narrow, W.draw_params(narrow, rng))
    assert B.nep_model_set_network(m8.handle, B.NEP_NETWORK_MFMA) == B.NEP_ERR_UNSUPPORTED
    assert B.nep_model_set_network(m8.handle, 7) == B.NEP_ERR_ARG
    assert B.nep_model_set_network(m8.handle, B.NEP_NETWORK_VALU) == B.NEP_OK
