"""The serving loop on the GPU: requests served in a mix (continuous
batching over several streams, admission by memory budget) give the same
structures and the same query answers as each request served alone."""
import numpy as np
import pytest

from tests.gpu_util import lib

pytestmark = pytest.mark.gpu


def _defined(s):
    bits, zeros, rd, s0, s1 = s.host_arrays()
    W = bits.shape[1]
    cap = -(-s.n // 4096) + 1
    return [bits, zeros, rd[:, : W // 8 + 1], s0[:, :cap], s1[:, :cap]]


def _trace(texts, n_req, seed):
    import torch
    from paper_1702_07578_amd import serving as S
    rng = np.random.default_rng(seed)
    reqs, builds, t = [], [], 0.0
    for rid in range(n_req):
        t += float(rng.exponential(0.0005))
        if builds and rng.random() < 0.4:
            target = int(rng.choice(builds))
            ti = reqs[target].text
            T, L = texts[ti]
            m = 4096
            op = int(rng.integers(0, 3))
            pos = rng.integers(0, T.size, size=m, dtype=np.int64)
            sym = T[pos].astype(np.int32)
            if rng.random() < 0.5:
                # inputs drawn on the device at launch (positions, symbols,
                # and k = rank + 1 for select)
                args = S.QuerySpec(m=m, seed=1000 + rid)
            elif op == S.ACCESS:
                args = (torch.from_numpy(pos).cuda(),)
            elif op == S.RANK:
                args = (torch.from_numpy(sym).cuda(), torch.from_numpy(pos).cuda())
            else:
                args = (torch.from_numpy(sym).cuda(), torch.ones(m, dtype=torch.int64).cuda())
            reqs.append(S.Request(rid=rid, kind=S.QUERY, arrival=t, target=target, op=op, args=args))
        else:
            ti = int(rng.integers(0, len(texts)))
            reqs.append(S.Request(rid=rid, kind=S.BUILD, arrival=t, text=ti, tree=int(rng.integers(0, 2))))
            builds.append(rid)
    return reqs


def _texts():
    from paper_1702_07578_amd import inputs
    out = []
    for i, (n, sigma) in enumerate([(5000, 256), (70000, 256), (200000, 1 << 16), (1 << 16, 4),
                                    (123457, 1 << 16), (3000, 1 << 16)]):
        T = inputs.uniform(n, sigma, 1 if sigma <= 256 else 2, 100 + i)
        out.append((T, inputs.lg_sigma(sigma)))
    return out


@pytest.mark.parametrize("slots,budget", [(4, 4 << 30), (2, 2 << 20)])
def test_mix_equals_alone(slots, budget):
    import torch
    from paper_1702_07578_amd import serving as S
    B = lib()
    texts = _texts()
    d_texts = [(B.to_device(T), T.size, T.dtype.itemsize, L) for T, L in texts]
    reqs = _trace(texts, 48, seed=slots)
    ex = S.GpuExecutor(d_texts, slots)
    srv = S.Server(ex, budget, slots=slots)
    done = srv.run(reqs, stall_s=30.0)
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    assert srv.peak_bytes <= budget
    by = {r.rid: r for r in done}
    alone = {}
    for r in reqs:
        if r.kind != S.BUILD:
            continue
        d, n, b, L = d_texts[r.text]
        s = B.build(d, n, b, L, r.tree)
        torch.cuda.synchronize()
        alone[r.rid] = s
        assert by[r.rid].status == 0
        if r.rid in srv.resident:
            for x, y in zip(_defined(srv.resident[r.rid][0]), _defined(s)):
                assert np.array_equal(x, y), f"build {r.rid}"
    answered = 0
    for r in reqs:
        if r.kind != S.QUERY or by[r.rid].status != 0:
            continue
        s = alone[r.target]
        inputs = by[r.rid].inputs
        if r.op == S.ACCESS:
            want = s.access(*inputs)
        elif r.op == S.RANK:
            want = s.rank(*inputs)
        else:
            want = s.select(*inputs)
        assert torch.equal(by[r.rid].result, want), f"query {r.rid}"
        if isinstance(r.args, S.QuerySpec):
            # drawn inputs: select answers the drawn positions, access the text
            T, _ = texts[reqs[r.target].text]
            if r.op == S.ACCESS:
                assert np.array_equal(want.cpu().numpy().astype(np.int64),
                                      T[inputs[0].cpu().numpy()].astype(np.int64))
            elif r.op == S.SELECT:
                ranks = s.rank(inputs[0], want)
                assert torch.equal(ranks + 1, inputs[1]), f"query {r.rid}: rank(select(k)) != k - 1"
        answered += 1
    assert answered > 0
    if budget == 2 << 20:
        assert srv.evictions > 0
    st = srv.stats()
    assert st["refused"] + st["lost_queries"] == sum(r.status != 0 for r in done)
