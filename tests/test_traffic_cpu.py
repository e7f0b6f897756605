"""CPU: the builder of profiles/traffic.json turns FETCH_SIZE / WRITE_SIZE per dispatch
(KiB, as the counter runs store them) into bytes per launch, each scaled by what the
same counter reads for the 256 MiB reference copy, and records the kernel-source hash
that bench.py checks before using the figures."""
import sqlite3

import pytest

from paper_2006_00686_amd import traffic


def _db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", [(k, counter, v) for k, v in rows])
    con.commit()
    con.close()


def test_scaled_bytes_per_launch(tmp_path):
    fetch, write = str(tmp_path / "fetch.db"), str(tmp_path / "write.db")
    fwd = "void xrt::(anonymous namespace)::k_forward<3, 1>(xrt::DevPlan, float const*)"
    att = "void xrt::(anonymous namespace)::k_forward_att<3, 1>(xrt::DevPlan, float const*)"
    fwd2 = "void xrt::(anonymous namespace)::k_forward<2, 1, false>(xrt::DevPlan, float const*)"
    gat = "void xrt::(anonymous namespace)::k_cone_gather<4, 3, false, false>(xrt::DevPlan)"
    # the reference copy reads half of its 256 MiB in FETCH_SIZE units and writes all of
    # it; the runtime's small copies must not be taken for it
    _db(fetch, "FETCH_SIZE", [(fwd, 1000.0), (fwd, 3000.0), (att, 9e9), (fwd2, 7e9), (gat, 500.0),
                              ("__amd_rocclr_copyBuffer", 4.0), ("__amd_rocclr_copyBuffer", 131072.0)])
    _db(write, "WRITE_SIZE", [(fwd, 10.0), (gat, 20.0), ("__amd_rocclr_copyBuffer", 262144.0)])
    t = traffic.build(fetch, write)
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    k = t["kernels"]["k_forward"]
    assert k["fetch_bytes"] == 2000 * 1024 * 2 and k["write_bytes"] == 10 * 1024
    assert k["bytes_per_launch"] == k["fetch_bytes"] + k["write_bytes"]
    assert t["kernels"]["k_cone_gather"]["bytes_per_launch"] == 500 * 1024 * 2 + 20 * 1024
    import bench
    assert t["source_hash"] == bench.kernel_source_hash()


def test_missing_reference_copy_is_an_error(tmp_path):
    fetch, write = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    _db(fetch, "FETCH_SIZE", [("k_forward<3, 1>", 1.0)])
    _db(write, "WRITE_SIZE", [("k_forward<3, 1>", 1.0)])
    with pytest.raises(SystemExit):
        traffic.build(fetch, write)


def test_a_copy_other_than_the_reference_is_rejected(tmp_path):
    fetch, write = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    fwd = "void xrt::(anonymous namespace)::k_forward<3, 1>(xrt::DevPlan)"
    _db(fetch, "FETCH_SIZE", [(fwd, 1.0), ("__amd_rocclr_copyBuffer", 524288.0)])
    _db(write, "WRITE_SIZE", [(fwd, 1.0), ("__amd_rocclr_copyBuffer", 1048576.0)])   # a 1 GiB copy
    with pytest.raises(SystemExit):
        traffic.build(fetch, write)
