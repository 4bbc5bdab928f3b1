"""The build refuses kernels that use scratch (private) memory: the parser of
hipcc's resource-usage remarks finds them (CPU only, no compilation)."""
import importlib.util
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SPEC = importlib.util.spec_from_file_location(
    "_build", os.path.join(HERE, "..", "paper_2511_15028_amd", "_build.py"))
B = importlib.util.module_from_spec(SPEC)
SPEC.loader.exec_module(B)

REMARKS = """\
x.hip:10:1: remark: Function Name: _Z5k_onePf [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     VGPRs: 12 [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark: Function Name: _Z5k_twoPf [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark:     ScratchSize [bytes/lane]: 32 [-Rpass-analysis=kernel-resource-usage]
x.hip:30:1: remark: Function Name: _Z7k_threePf [-Rpass-analysis=kernel-resource-usage]
x.hip:30:1: remark:     ScratchSize [bytes/lane]: 4 [-Rpass-analysis=kernel-resource-usage]
"""


def test_scratch_kernels_are_found():
    assert B._scratch_kernels(REMARKS) == [("_Z5k_twoPf", 32), ("_Z7k_threePf", 4)]


def test_no_scratch_no_report():
    assert B._scratch_kernels(REMARKS.split("x.hip:20")[0]) == []
