"""Autotune tables as text (host logic, no GPU): load, report, save, and the
rejection of malformed tables and bad modes."""
import pytest

from paper_2503_16225_amd import binding as B


def test_table_round_trip(tmp_path):
    lib = B.load_library()
    src = tmp_path / "t.txt"
    src.write_text("# comment\n"
                   "gfx950/256 gemm_hn f32 n98304 a1536 b512: choice 4 ms 4.5 5.0 4.9 6.2 4.0 7.6\n"
                   "gfx950/256 gemm_nn f32 n98304 a3072 b512: choice 1 ms 6.0 5.5\n"
                   "\n")
    assert B.autotune_load(src) == 2
    assert B.autotune_load(src) == 0  # entries already present are kept
    rep = B.autotune_report()
    assert "gfx950/256 gemm_hn f32 n98304 a1536 b512: choice 4 ms 4.5 5 4.9 6.2 4 7.6" in rep
    assert "gfx950/256 gemm_nn f32 n98304 a3072 b512: choice 1 ms 6 5.5" in rep
    out = tmp_path / "saved.txt"
    B.autotune_save(out)
    assert out.read_text() == rep
    assert lib.eahp_autotune_enable(3) == -1  # EAHP_EINVAL


@pytest.mark.parametrize("line", ["gfx950/256 gemm_hn f32 n1 a1 b1 choice 2\n",
                                  "gfx950/256 gemm_hn f32 n1 a1 b1: choice x\n",
                                  "gfx950/256 gemm_hn f32 n1 a1 b1: choice -1\n"])
def test_malformed_table_rejected(tmp_path, line):
    bad = tmp_path / "bad.txt"
    bad.write_text(line)
    with pytest.raises(B.EahpError):
        B.autotune_load(bad)


def test_missing_table_rejected(tmp_path):
    with pytest.raises(B.EahpError):
        B.autotune_load(tmp_path / "none.txt")
