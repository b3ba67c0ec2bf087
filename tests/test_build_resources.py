"""The build's per-kernel resource table: every HIP kernel runs without
private (scratch) memory.  A large private segment per lane once made the
queue refuse a dispatch at run time; the build now refuses such a kernel
instead, and this checks the table the last build wrote."""
import json
import os

import pytest

from paper_2604_12256_amd import build as B


def test_resource_table_has_no_scratch():
    if not os.path.exists(B.RESOURCES):
        pytest.fail(f"{B.RESOURCES} missing: run the build (python -m paper_2604_12256_amd.build)")
    with open(B.RESOURCES) as f:
        table = json.load(f)
    names = " ".join(table)
    for kernel in ("k_stage", "k_dense", "k_dense_mfma", "k_diag", "k_kron", "k_small", "k_marg_partial",
                   "k_inner_partial", "k_sample", "k_expect_z_partial", "k_collapse", "k_copy"):
        assert kernel in names, kernel
    assert B.scratch_offenders(table) == []
    for f, r in table.items():
        assert r["ScratchSize [bytes/lane]"] == 0, f
        assert r["VGPRs Spill"] == 0, f


def test_parser_flags_a_kernel_with_scratch():
    text = "\n".join([
        "a.hip:1:1: remark: Function Name: k_good [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     VGPRs: 24 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     Dynamic Stack: False [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark: Function Name: k_spills [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     VGPRs: 256 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     ScratchSize [bytes/lane]: 18272 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     Dynamic Stack: False [-Rpass-analysis=kernel-resource-usage]",
    ])
    t = B.parse_resource_report(text)
    assert t["k_good"]["VGPRs"] == 24 and t["k_spills"]["ScratchSize [bytes/lane]"] == 18272
    assert B.scratch_offenders(t) == ["k_spills"]
