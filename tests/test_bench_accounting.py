"""The benchmark's algorithmic byte counts (the roofline numerator) against
the per-array sums written out by hand for the Taylor-Green workload."""
import bench


def test_flux_kernel_bytes_taylor_green_fp32():
    nc, nf = 288 ** 3, 3 * 288 ** 3
    total, per_cell, per_face = bench.flux_kernel_bytes(nc, nf, 5, 3, 4, "USR5", blend=True)
    # per cell: U 20 + G1 60 + 1/V 4 + slot_ptr 4 + R/U out 20 + 2/3 of U^n 20 + theta 4
    assert abs(per_cell - (20 + 60 + 4 + 4 + 20 + 20 * 2 / 3 + 4)) < 1e-9
    # per face: owner/neighbour 8 + S, omega 16 + d 12 + two slots 4 + record positions 2 + d.H.d of both
    # cells 40
    assert per_face == 8 + 16 + 12 + 4 + 2 + 40
    assert abs(total - (9.013690368e9 - 2 * nf)) < 1.0


def test_flux_kernel_bytes_fp64():
    _t, per_cell, per_face = bench.flux_kernel_bytes(1, 1, 5, 3, 8, "USR5", blend=True)
    # FP64: d (3 doubles); the coefficients are evaluated in the kernel
    assert per_face == 8 + 32 + 3 * 8 + 4 + 2 + 80
    assert abs(per_cell - (40 + 120 + 8 + 4 + 40 + 40 * 2 / 3 + 4)) < 1e-9


def test_gradient_kernel_bytes_taylor_green_fp32():
    nc = 288 ** 3
    nrec = 6 * nc  # six face records per hexahedron
    # per cell: U 20 + 1/V 4 + face count 4 + G1 60 + features 48; per record: 16 + 12 bytes of records
    assert bench.grad_features_bytes(nc, nrec, 5, 3, 4) == nc * (20 + 4 + 4 + 60 + 48) + nrec * 28
    # plain gradient: U 20 + 1/V 4 + G1 60 per cell, sigma w S and the other cell (16) per record
    assert bench.grad_bytes(nc, nrec, 5, 3, 4) == nc * (20 + 4 + 60) + nrec * 16
    # per cell: G1 60 + 1/V 4 + face count 4; per record: records 28 + d.H.d 20
    assert bench.hface_bytes(nc, nrec, 5, 3, 4) == nc * (60 + 4 + 4) + nrec * (28 + 20)
    assert bench.COMPULSORY_BYTES["fp32"] == 360 and bench.COMPULSORY_BYTES["fp64"] == 504


def test_committed_counter_summaries_belong_to_the_current_kernels():
    """The rocprofv3 summaries under profiles/ that the benchmark and the
    design notes quote were taken on kernels whose code (comments stripped)
    hashes to the current sources: the traffic summary (read back into the
    bench line's roofline) and the vector-issue / address-unit summary."""
    import os
    import re
    from paper_2404_08952_amd import profiling
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cur = profiling.source_hash()
    got = profiling.read_summary(os.path.join(root, "profiles", "stage_kernels_tgv288_usr5_hllc_learned.txt"))
    assert got is not None and got[1] == cur
    assert len(bench.measured_traffic("tgv3d")) == 7
    with open(os.path.join(root, "profiles", "stage_kernels_tgv288_busy.txt")) as fh:
        m = re.search(r"kernel_source_sha256\s*=\s*(\S+)", fh.read())
    assert m is not None and m.group(1) == cur
