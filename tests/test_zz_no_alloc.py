"""lsim_decode_noalloc (the decode entry point that allocates nothing) gives
the same bits and posteriors as lsim_decode with a caller workspace, on two
calls in a row (the second on a smaller batch, so the scratch holds the
first call's state), and rejects a batch whose layered-decoder state would
not fit its static scratch before launching anything."""
import numpy as np
import pytest
import torch

import paper_2203_11854_amd as L
from helpers import graph, oracle_llrs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SCRATCH = 64 << 20


def _llrs(name, B, ebn0, seed):
    tx = oracle_llrs(name, B, ebn0, seed)
    return torch.from_numpy(tx["L"].astype(np.float32)).to(DEV)


def _both(code, llr, p):
    B = llr.shape[0]
    ref_bits, ref_app = L.decode(code, llr, p, want_app=True)
    bits = torch.full((B, code.k), 7, dtype=torch.uint8, device=DEV)
    app = torch.full((B, code.n_dec), float("nan"), dtype=torch.float32, device=DEV)
    L.decode_noalloc(code, llr, p, bits, app)
    torch.cuda.synchronize()
    return ref_bits, ref_app, bits, app


@pytest.mark.parametrize("name,B1,B2,ebn0", [("bg2", 300, 37, 1.5), ("bg1", 160, 9, 2.5)])
def test_noalloc_layered_equals_decode_twice(name, B1, B2, ebn0):
    qb, g = graph(name)
    code = L.Code.from_qcbase(qb, g.e_tx)
    p = L.params(L.NMS_F32, iters=20, alpha=0.75)
    assert L.decode_workspace(code, p, B1) <= SCRATCH
    for B, seed in ((B1, 0x2203118500000311), (B2, 0x2203118500000312)):
        print(f"[noalloc] {name} B={B} seed={seed:#x}", flush=True)
        llr = _llrs(name, B, ebn0, seed)
        rb, ra, b, a = _both(code, llr, p)
        assert torch.equal(b, rb), f"{name} B={B}: bits differ"
        assert torch.equal(a, ra), f"{name} B={B}: posteriors differ"


def test_noalloc_flooding_pass_through():
    qb, g = graph("bg2")
    code = L.Code.from_qcbase(qb, g.e_tx)
    llr = _llrs("bg2", 40, 2.5, 0x2203118500000313)
    for p, x in ((L.params(L.SPA_F32), llr), (L.params(L.OMS_I8), L.quantize(llr))):
        print(f"[noalloc] flooding algo={p.algo}", flush=True)
        rb, ra, b, a = _both(code, x, p)
        assert torch.equal(b, rb) and torch.equal(a, ra)


def test_noalloc_rejects_a_batch_beyond_the_scratch():
    qb, g = graph("bg1")
    code = L.Code.from_qcbase(qb, g.e_tx)
    p = L.params(L.NMS_F32)
    per_cw = L.decode_workspace(code, p, 1)
    B = SCRATCH // per_cw + 1
    assert L.decode_workspace(code, p, B) > SCRATCH
    llr = torch.zeros((B, g.e_tx), dtype=torch.float32, device=DEV)
    bits = torch.zeros((B, code.k), dtype=torch.uint8, device=DEV)
    with pytest.raises(L.LsimError, match="status 2.*scratch"):
        L.decode_noalloc(code, llr, p, bits)
    # the largest batch that fits still decodes
    Bmax = SCRATCH // per_cw
    print(f"[noalloc] bg1 largest batch B={Bmax}", flush=True)
    L.decode_noalloc(code, llr[:Bmax], p, bits[:Bmax])
    torch.cuda.synchronize()
    assert int(bits[:Bmax].sum()) == 0   # all-zero LLRs decode to the zero word
