"""Build-level checks that need no GPU: the HIP sources cross-compile for
gfx950, and no kernel spills registers to scratch memory (a spill is device
memory traffic on the hot path)."""

import os
import re
import shutil
import subprocess

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_2406_15186_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not installed")
@pytest.mark.parametrize("src", ["bank.hip", "stream.hip", "signif.hip", "harmonic.hip"])
def test_kernels_do_not_spill(tmp_path, src):
    from paper_2406_15186_amd.build import EXTRA, FLAGS
    cmd = ["hipcc", *FLAGS, *EXTRA.get(src, []), "-Rpass-analysis=kernel-resource-usage", "-c",
           os.path.join(CSRC, src), "-o", str(tmp_path / "k.o")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", r.stderr)
    scratch = [int(v) for v in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    assert names and len(names) == len(scratch)
    spilled = [(n, s) for n, s in zip(names, scratch) if s]
    assert not spilled, spilled
