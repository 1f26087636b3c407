"""The no-allocation evaluation entry point (qqa_dev_eval_noalloc) against qqa_dev_eval,
through the C ABI: identical integers on two calls in a row, the second on a smaller
input (the fixed scratch keeps the first call's contents and must be cleared)."""

import numpy as np
import pytest

import qqa_inputs as qi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _graph(problem, n, d, seed):
    g = qi.erdos_renyi(n, d, seed)
    return qi.pm1_weights(g, seed + 1) if problem == "maxcut" else g


def _state(n, S, stride, seed):
    rng = np.random.default_rng(seed)
    vals = np.array([0.0, 1.0, 0.5, np.nextafter(np.float32(0.5), np.float32(1)), 0.25, 0.75], np.float32)
    P = np.zeros((n, stride), np.float32)
    P[:, :S] = rng.choice(vals, size=(n, S), p=[0.35, 0.35, 0.1, 0.1, 0.05, 0.05])
    return P


def _eval(q, fn, G, problem, S, P):
    d = torch.device("cuda")
    out = [torch.full((S,), -99, dtype=torch.int64, device=d) for _ in range(3)]
    best = torch.full((1,), -5, dtype=torch.int32, device=d)
    fn(G, problem, 2, S, torch.as_tensor(P, device=d), *out, best)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out] + [int(best.item())]


@pytest.mark.parametrize("problem", ["mis", "maxcut", "maxclique"])
def test_noalloc_eval_equals_eval_on_two_calls(problem):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_02135_amd as q
    cases = [(_graph(problem, 3000, 8.0, 1), 1000), (_graph(problem, 300, 5.0, 2), 13)]
    for k, (g, S) in enumerate(cases):
        stride = q.qqa_replica_stride(S)
        P = _state(g["n"], S, stride, 10 + k)
        G = q.DevGraph(g)
        ref = _eval(q, q.qqa_dev_eval, G, problem, S, P)
        got = _eval(q, q.qqa_dev_eval_noalloc, G, problem, S, P)
        print(problem, g["n"], S, "best", ref[3], got[3], flush=True)
        for a, b in zip(ref[:3], got[:3]):
            assert np.array_equal(a, b)
        assert ref[3] == got[3]


def test_noalloc_eval_largest_stride_and_refusals():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_02135_amd as q
    g = _graph("mis", 200, 4.0, 3)
    S = 4096
    P = _state(g["n"], S, q.qqa_replica_stride(S), 4)
    G = q.DevGraph(g)
    ref = _eval(q, q.qqa_dev_eval, G, "mis", S, P)
    got = _eval(q, q.qqa_dev_eval_noalloc, G, "mis", S, P)
    for a, b in zip(ref[:3], got[:3]):
        assert np.array_equal(a, b)
    assert ref[3] == got[3]
    # S beyond the maximum is refused before any launch
    d = torch.device("cuda")
    with pytest.raises(q.QQAError):
        out = torch.zeros(4097, dtype=torch.int64, device=d)
        q.qqa_dev_eval_noalloc(G, "mis", 2, 4097, torch.zeros((g["n"], 4100), device=d), out, out.clone(),
                               out.clone(), torch.zeros(1, dtype=torch.int32, device=d))
