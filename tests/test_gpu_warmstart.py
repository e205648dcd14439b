"""The learned warm start inside the solver: the energy judge, through the C ABI.

The judge evaluates the energy at the previous frame's result and at the
network's prediction and keeps the lower as the frame's start.  Checked here:
it keeps the previous start for a network that predicts no change and for one
that predicts garbage (results bitwise equal to a solve without a network), it
takes a prediction that is better (results bitwise equal to a plain solve
started from that prediction), and the energies it compares match the oracle's
energy of the same states.
"""
import sys

import numpy as np
import pytest

import oracle as O
from oracle.energy import prepare_frame, total_energy
from scenes import make_clip

pytestmark = pytest.mark.gpu
P32 = O.default_params(state_precision="f32")


def _say(*m):
    print("[gpu-case]", *m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_01961_amd as G
    G.load_library()
    return _t


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _flat_zero(K):
    import paper_1908_01961_amd as G
    return np.zeros(int(G.load_library().gid_net_num_params(K)), np.float32)


def _out_bias_index(K, channel):
    """Index of the output layer's bias for one output channel in the parameter vector."""
    n = K + 4
    cin = [3 + n] + [32] * 5
    cout = [32] * 5 + [n]
    off = 0
    for l in range(6):
        off += cout[l] * cin[l] * 9
        if l == 5:
            return off + channel
        off += cout[l]


CLIP = dict(W=96, H=64, K=4, F=3, seed=515)


def _setup(torch, net_params=None, corrupt=0.0):
    """Solver loaded with the oracle's frame-0 result (T_0 shifted by `corrupt`)
    as the previous frame; returns the solver, the clip and that state."""
    import paper_1908_01961_amd as G
    c = make_clip(CLIP["W"], CLIP["H"], CLIP["K"], CLIP["F"], CLIP["seed"])
    f0 = O.decompose_clip(c.frames, c.ids, c.b_init, P32, 3, 8, temporal=True, nframes=1)[0]
    u32 = f0.u.astype(np.float32)
    u_start = u32.copy()
    u_start[3] += np.float32(corrupt)
    s = G.Solver(c.width, c.height, G.default_params(c.K, gn_iters=2, pcg_iters=6, temporal=1, record_energy=1))
    s.set_base_colors(c.b_init)
    s.set_prev_frame(_dev(torch, c.frames[0]), _dev(torch, u32[:3]))
    s.set_state(_dev(torch, u_start), f0.b)
    net = None
    if net_params is not None:
        net = G.Net(c.K, c.width, c.height)
        net.set_params(net_params)
        s.set_warmstart(net)
    return s, net, c, f0, u_start


def _solve(torch, s, c, t=1):
    lay = torch.empty((c.K + 4, c.height, c.width), dtype=torch.float32, device="cuda")
    b, st = s.decompose_frame(_dev(torch, c.frames[t]), _dev(torch, c.ids[t]), lay)
    return lay.cpu().numpy(), b, st


def test_identity_network_keeps_the_previous_start(torch):
    s0, _, c, _, _ = _setup(torch)
    L0, b0, st0 = _solve(torch, s0, c)
    s1, net, _, _, _ = _setup(torch, _flat_zero(c.K))
    L1, b1, st1 = _solve(torch, s1, c)
    _say(f"identity network: judged {st1['warm_start_learned']}, E prev {st1['energy_start_previous']:.9e} "
         f"E net {st1['energy_start_learned']:.9e}")
    assert st0["warm_start_learned"] == -1 and st1["warm_start_learned"] == 0
    assert st1["energy_start_learned"] == st1["energy_start_previous"]
    assert np.array_equal(L0, L1) and np.array_equal(b0, b1) and st0["energy_final"] == st1["energy_final"]
    s0.close(); s1.close(); net.close()


def test_garbage_network_is_rejected(torch):
    rng = np.random.default_rng(3)
    flat = (rng.normal(0.0, 3.0, size=_flat_zero(CLIP["K"]).size)).astype(np.float32)
    s0, _, c, _, _ = _setup(torch)
    L0, b0, st0 = _solve(torch, s0, c)
    s1, net, _, _, _ = _setup(torch, flat)
    L1, b1, st1 = _solve(torch, s1, c)
    _say(f"garbage network: judged {st1['warm_start_learned']}, E prev {st1['energy_start_previous']:.6e} "
         f"E net {st1['energy_start_learned']:.6e}")
    assert st1["warm_start_learned"] == 0
    assert not (st1["energy_start_learned"] < st1["energy_start_previous"])
    assert np.array_equal(L0, L1) and np.array_equal(b0, b1)
    s0.close(); s1.close(); net.close()


def test_better_prediction_is_taken_and_energies_match_the_oracle(torch):
    import paper_1908_01961_amd as G
    K = CLIP["K"]
    flat = _flat_zero(K)
    flat[_out_bias_index(K, 3)] = -0.1                   # the network moves T_0 back by 0.1
    s1, net, c, f0, u_start = _setup(torch, flat, corrupt=0.1)
    L1, b1, st1 = _solve(torch, s1, c)
    _say(f"corrected start: judged {st1['warm_start_learned']}, E prev {st1['energy_start_previous']:.9e} "
         f"E net {st1['energy_start_learned']:.9e}")
    assert st1["warm_start_learned"] == 1
    assert st1["energy_start_learned"] < st1["energy_start_previous"]
    # the judge's energies are the oracle's energies of the two starts
    fd = prepare_frame(c.frames[1], c.ids[1], P32, f0.fd.C, f0.u[:3].astype(np.float32).astype(np.float64))
    e_prev = total_energy(u_start.astype(np.float64), f0.b, fd, P32)
    # with every other parameter zero the trunk's features are zero: du is the output bias alone
    u_net = u_start.astype(np.float64).copy()
    u_net[3] = (u_start[3] + np.float32(-0.1)).astype(np.float64)
    e_net = total_energy(u_net, f0.b, fd, P32)
    _say(f"oracle: E prev {e_prev:.9e}, E net {e_net:.9e}")
    assert st1["energy_start_previous"] == pytest.approx(e_prev, rel=1e-9)
    assert st1["energy_start_learned"] == pytest.approx(e_net, rel=1e-9)
    # the rest of the frame is the plain schedule from the prediction
    s2, _, _, _, _ = _setup(torch)
    s2.set_state(_dev(torch, u_net.astype(np.float32)), f0.b)
    L2, b2, st2 = _solve(torch, s2, c)
    assert np.array_equal(L1, L2) and np.array_equal(b1, b2) and st1["energy_final"] == st2["energy_final"]
    s1.close(); s2.close(); net.close()


def test_first_frame_is_not_judged_and_batches_refuse_a_network(torch):
    import paper_1908_01961_amd as G
    c = make_clip(64, 32, 3, 2, 9)
    s = G.Solver(64, 32, G.default_params(3, gn_iters=1, pcg_iters=4))
    s.set_base_colors(c.b_init)
    net = G.Net(3, 64, 32)
    net.set_params(_flat_zero(3))
    s.set_warmstart(net)
    _, _, st = _solve(torch, s, c, t=0)
    assert st["warm_start_learned"] == -1 and np.isnan(st["energy_start_learned"])
    with pytest.raises(G.GidError) as ei:
        G.Batch([s]).step([_dev(torch, c.frames[1])], [_dev(torch, c.ids[1])])
    assert ei.value.status == 6
    other = G.Net(3, 32, 32)
    with pytest.raises(G.GidError):
        s.set_warmstart(other)
    s.close(); net.close(); other.close()
