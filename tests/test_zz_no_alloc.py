"""The refinement entry point that allocates nothing (hgp_refine_lp_static)
against the workspace entry point (hgp_refine_lp) through the C ABI: two
calls in a row on one device, the second on a smaller input, so the second
call finds the first call's contents in the shared scratch array."""
import sys

import numpy as np
import pytest

from paper_2303_17679_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_static_scratch_matches_workspace_entry_point(orc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_17679_amd as H
    H.lib()
    cases = [(W.random_uniform(60000, 60000, 2, 8, seed=3), 16, 4),
             (W.random_uniform(3000, 2500, 2, 6, seed=8), 4, 9)]
    for h, k, seed in cases:
        print(f"[no-alloc] n={h.n} m={h.m} k={k}", file=sys.stderr, flush=True)
        P = H.params(k, seed=seed)
        G = H.Hypergraph.from_host(h)
        part0 = orc.greedy_ip(h, k)
        t_ws = torch.from_numpy(part0.view(np.int32)).cuda()
        t_st = t_ws.clone()
        f_ws, bw_ws = H.refine_lp(G, P, 1, t_ws)
        f_st, bw_st = H.refine_lp_static(G, P, 1, t_st)
        torch.cuda.synchronize()
        assert f_st == f_ws
        assert torch.equal(t_st, t_ws)
        assert torch.equal(bw_st, bw_ws)
        out_o, f_o, bw_o, _, _ = orc.refine_lp(h, orc.params(k, seed=seed), 1, part0)
        assert f_st == f_o and np.array_equal(t_st.cpu().numpy().view(np.uint32), out_o)
