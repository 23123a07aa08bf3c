"""The profile summariser on small synthetic rocprofv3 CSV outputs: the
counter scale comes from the bandwidth probe's copy kernel, read bytes from
the read requests by size where they were taken, and the per-storage bytes
per launch feed the bench's roofline.traffic."""
import csv
import json
import os

import pytest

from paper_2110_13055_amd import profile_summary as ps

NF = 1000
FUSED32 = "void cdi::(anonymous namespace)::step_kernel<cdi::D3Q19, 0, 2, 1, 1>(cdi::Grid, cdi::Phys, cdi::Bufs)"
LBM16 = "void cdi::(anonymous namespace)::step_kernel<cdi::D3Q19, 3, 2, 1, 0>(cdi::Grid, cdi::Phys, cdi::Bufs)"
COPY = "void cdi::(anonymous namespace)::copy_kernel(uint4 const*, uint4*, unsigned long)"
MIB = 4


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def _counters(d, rows):
    _write(os.path.join(d, "run_counter_collection.csv"),
           ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)


@pytest.fixture
def runs(tmp_path):
    t = str(tmp_path)
    _write(os.path.join(t, "trace", "run_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
           [[FUSED32, 2, 4000, 2000.0, 50, 2000, 2000, 0], [LBM16, 2, 2000, 1000.0, 25, 1000, 1000, 0]])
    copy = MIB * 1024 * 1024
    # FETCH_SIZE in KiB units counting each 128-byte read as 64 bytes: half the copy
    _counters(os.path.join(t, "fetch"), [[1, COPY, "FETCH_SIZE", copy / 2048],
                                         [2, FUSED32, "FETCH_SIZE", 150 * NF / 2048],
                                         [3, FUSED32, "FETCH_SIZE", 150 * NF / 2048],
                                         [4, LBM16, "FETCH_SIZE", 60 * NF / 2048]])
    _counters(os.path.join(t, "write"), [[1, COPY, "WRITE_SIZE", copy / 1024],
                                         [2, FUSED32, "WRITE_SIZE", 100 * NF / 1024],
                                         [4, LBM16, "WRITE_SIZE", 40 * NF / 1024]])
    # exact reads: the fused kernel 140 B/node as 128- and 64-byte requests
    _counters(os.path.join(t, "rdreq"), [[2, FUSED32, "TCC_EA0_RDREQ_128B", 128 * NF / 128],
                                         [2, FUSED32, "TCC_EA0_RDREQ_64B", 12 * NF / 64],
                                         [2, FUSED32, "TCC_EA0_RDREQ_32B", 0]])
    with open(os.path.join(t, "bench.log"), "w") as fh:
        fh.write(json.dumps({"metric": "m", "config": {"n_fluid": NF}}) + "\n")
    return t


def test_scales_and_per_node_bytes(runs):
    rec, md = ps.summarise(os.path.join(runs, "trace"), os.path.join(runs, "fetch"), os.path.join(runs, "write"),
                           os.path.join(runs, "bench.log"), MIB, ["cmd"], os.path.join(runs, "rdreq"))
    assert rec["counter_scale"] == {"FETCH_SIZE": 2048.0, "WRITE_SIZE": 1024.0}
    rows = {r["kernel"]: r for r in rec["kernels"]}
    f = rows["D3Q19 fp32 fused pull"]
    assert f["read_per_node"] == pytest.approx(140.0)          # from the requests
    assert f["fetch_scaled_per_node"] == pytest.approx(150.0)  # FETCH_SIZE x scale, shown beside
    assert f["write_per_node"] == pytest.approx(100.0)
    assert f["gbs"] == pytest.approx(240.0 * NF / 2e-6 / 1e9)
    l16 = rows["D3Q19 fp16 lbm pull"]                          # no request counts: FETCH_SIZE x scale
    assert l16["read_per_node"] == pytest.approx(60.0) and l16["write_per_node"] == pytest.approx(40.0)
    assert rec["bytes_per_launch"]["fp32"] == pytest.approx(240.0 * NF)
    assert rec["lbm_bytes_per_launch"]["fp16"] == pytest.approx(100.0 * NF)
    assert rec["kernel_source_hash"] == ps.kernel_source_hash()
    assert "| D3Q19 fp32 fused pull | 2 | 0.002 | 140.0 | 150.0 | 100.0 |" in md


def test_variant_labels():
    assert ps._variant(FUSED32) == "D3Q19 fp32 fused pull"
    assert ps._variant(LBM16) == "D3Q19 fp16 lbm pull"
    assert ps._variant("void cdi::(anonymous namespace)::step_kernel<cdi::D3Q19, 2, 0, 1, 1>(x)") == "D3Q19 moments fused"
    assert ps._variant("void cdi::(anonymous namespace)::step_kernel<cdi::D2Q9, 0, 0, 0, 1>(x)") == "D2Q9 fp32 np"
    # the sixth argument: the odd step staged in LDS
    assert (ps._variant("void cdi::(anonymous namespace)::step_kernel<cdi::D3Q19, 0, 1, 1, 1, 1>(x)")
            == "D3Q19 fp32 fused odd staged")
    assert ps._variant("void cdi::(anonymous namespace)::step_kernel<cdi::D3Q19, 0, 0, 1, 1, 0>(x)") == \
        "D3Q19 fp32 fused even"
    assert ps._variant(COPY) is None
