"""The product path has no CPU fallback: without a GPU every compute entry of
the binding raises, and a missing library raises at load instead of routing
anywhere else."""
import pytest

rtq = pytest.importorskip("paper_2001_02620_amd")
torch = pytest.importorskip("torch")

from paper_2001_02620_amd import scenegen as sg  # noqa: E402


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the behaviour on a host without a GPU")
def test_compute_entries_raise_without_gpu():
    scene = sg.tiny_scene(1)
    with pytest.raises(RuntimeError, match="GPU"):
        rtq.Scene(scene)


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(rtq, "_lib", None)
    monkeypatch.setattr(rtq, "LIB_PATH", str(tmp_path / "librtq.so"))
    with pytest.raises(ImportError, match="not built"):
        rtq.load_library()
