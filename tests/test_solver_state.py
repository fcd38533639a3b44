"""CPU: the iterate state of the reconstruction loops (section IV's x_k,
y_k, t_k; section V's K_d, K_r and y-tilde) written by save_state reads
back unchanged with torch.load(weights_only=True)."""
import pytest

torch = pytest.importorskip("torch")

from paper_1603_02329_amd import solver as S  # noqa: E402


@pytest.mark.parametrize("mg", [False, True])
def test_state_roundtrip(mg, tmp_path):
    g = torch.Generator().manual_seed(5)
    x, y = torch.rand(8, 6, generator=g), torch.rand(8, 6, generator=g)
    if mg:
        hist = [S.MGRecord("direct", 1.5, 0, 0.1, 0, 0.25), S.MGRecord("recursive", 1.25, 3, 0.4, 2, 0.2)]
        st = S.IterState(2, x, y, 1.618, hist, 0, 1, torch.rand(8, 6, generator=g))
    else:
        st = S.IterState(4, x, y, 2.5, [3.0, 2.5, 2.25, 2.125])
    path = str(tmp_path / "s.pt")
    S.save_state(path, st)
    back = S.load_state(path, "cpu")
    assert back.k == st.k and back.t == st.t and back.k_d == st.k_d and back.k_r == st.k_r
    assert torch.equal(back.x_prev, x) and torch.equal(back.y, y)
    assert back.hist == st.hist
    assert (back.y_tilde is None) == (st.y_tilde is None)
    if mg:
        assert torch.equal(back.y_tilde, st.y_tilde)
