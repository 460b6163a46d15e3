"""Host-side admission logic of the serving loop (no GPU): a request whose
solver slot alone exceeds the memory budget is rejected instead of blocking
the first-in-first-out queue behind it."""
from paper_2609_04534_amd import serve, tpfdm


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


def test_every_class_of_the_serving_mix_uses_multigrid():
    """All 15 classes (p in {2, 3, 7}, m in {8, 16, 24, 32, 48}) have a
    coarsest level the library solves densely: at degree p for p <= 3, and
    for p = 7 either one cell (m a power of two) or the degree-1 level on
    3^3 cells (216 unknowns); larger odd parts are left to block-Jacobi."""
    for p in (2, 3, 7):
        for m in (8, 16, 24, 32, 48):
            assert serve.uses_multigrid(p, m), (p, m)
    assert not serve.uses_multigrid(7, 7)      # 343 cells: 2744 unknowns even at degree 1
    assert not serve.uses_multigrid(3, 5)      # 125 cells of degree 3 (lane kernels keep their degree)
    assert serve.uses_multigrid(4, 40)         # odd part 5: 125 cells x 8 = 1000


def test_multigrid_level_storage_follows_the_inner_precision():
    """Slots of an FP32-inner server keep FP32 multigrid level vectors, at
    half the bytes; an FP64-inner server FP64 ones."""
    for p in (2, 3, 7):
        assert serve.mg_storage(p, tpfdm.F32) == tpfdm.F32
        assert serve.mg_storage(p, tpfdm.F64) == tpfdm.F64
    assert 2 * serve.mg_bytes(7, 16, tpfdm.F32) == serve.mg_bytes(7, 16)
    assert 2 * serve.mg_bytes(3, 16, tpfdm.F32) == serve.mg_bytes(3, 16)
    assert (serve.class_slot_bytes(3, 16, True, tpfdm.F32) - serve.class_slot_bytes(3, 16)
            == serve.mg_bytes(3, 16, tpfdm.F32))
