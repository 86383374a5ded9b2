"""Host-side logic of bench.py that needs no GPU: the algorithmic byte models behind the
roofline figures and the kernel-source check that gates the counter-based traffic."""
import json

import pytest

import bench


def test_apply_bytes_per_pixel():
    # read k maps and k(k+1)/2 packed mixing planes, write k maps
    assert bench.apply_bytes_per_pixel(3, 4) == (3 + 6 + 3) * 4 == 48
    assert bench.apply_bytes_per_pixel(3, 8) == 96
    # where there are fewer weight maps than packed planes, the weights are the reads
    assert bench.apply_bytes_per_pixel(4, 4, f=9) == (4 + 9 + 4) * 4
    assert bench.apply_bytes_per_pixel(4, 4, f=20) == (4 + 10 + 4) * 4


@pytest.mark.parametrize("k,elem,expect", [
    # float32, k = 3: apply p_old, z, x, M32 in; p, q, x out = 6k + mk planes of 4 B;
    # update r, q in, r, z out (4k planes) + 6 bfloat16 planes
    (3, 4, (6 * 3 + 6) * 4 + 4 * 3 * 4 + 6 * 2),
    # float64, k = 3: x advanced every second iteration (1.5 k planes on average)
    (3, 8, (4 * 3 + 6 + 4.5) * 8 + 4 * 3 * 8 + 6 * 2),
    (4, 4, (6 * 4 + 10) * 4 + 4 * 4 * 4 + 10 * 2),
])
def test_cg_iteration_bytes_per_pixel(k, elem, expect):
    assert bench.cg_iteration_bytes_per_pixel(k, elem) == pytest.approx(expect)
    if (k, elem) == (3, 4):
        assert expect == 156
    if (k, elem) == (3, 8):
        assert expect == 288


def test_traffic_gated_by_kernel_source(tmp_path, monkeypatch):
    rec = tmp_path / "traffic.json"
    rec.write_text(json.dumps({"kernel_source_sha": "abc", "traffic_bytes_per_launch": 123}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    assert bench.traffic_from_counters("abc") == 123
    assert bench.traffic_from_counters("def") is None
    rec.write_text("not json")
    assert bench.traffic_from_counters("abc") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.traffic_from_counters("abc") is None


def test_more_than_one_gpu_refused(monkeypatch, capsys):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code != 0
    assert "one GPU" in capsys.readouterr().err
