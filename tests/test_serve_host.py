"""Host-side admission logic of the serving loop (no GPU): a request whose
solver slot alone exceeds the memory budget is rejected instead of blocking
the first-in-first-out queue behind it."""
from paper_2609_04534_amd import serve


def test_class_slot_bytes_matches_the_layout():
    # p = 3 (n = 4, B = 64): 8^3 = 512 cells -> 512 * 64 elements per vector
    E = 512 * 64
    assert serve.class_slot_bytes(3, 8) == 7 * E * 8 + 3 * 8 * 8 + 256
    # p = 7 (n = 8, B = 1): 3^3 cells
    E7 = 27 * 512
    assert serve.class_slot_bytes(7, 3) == 7 * E7 * 8 + 3 * 1 * 8 + 256
    assert serve.class_slot_bytes(3, 8, multigrid=True) > serve.class_slot_bytes(3, 8)


def test_oversized_requests_are_rejected_without_running():
    budget = serve.class_slot_bytes(2, 8) // 2
    reqs = [serve.Request(k, 2, 8, arrival=0.0, b=None) for k in range(3)]
    srv = serve.Server(hbm_budget=budget)
    done = srv.run(reqs)
    assert srv.rejected == 3 and not srv.busy and not srv.plans
    for r in done:
        assert r.rejected and r.x is None and r.summary["status"] == "rejected"
        assert "exceeds the budget" in r.summary["reason"]
