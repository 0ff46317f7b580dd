"""Static check of the gfx950 assembly of the chain kernel and of the 3x3
reflector sweep (CPU only).

Both sweeps read coefficients through DPP (row_newbcast) operands written in
inline assembly, where the compiler cannot insert the two wait states the
hardware needs between a VALU write of a VGPR and a DPP read of it.  The
kernel is built so that every DPP source is written by a memory load; this
test compiles the kernel to assembly and checks that no DPP source register
was written by a VALU instruction in the two preceding instructions, and
that no sweep kernel spills registers to scratch memory.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_01852_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def vregs(text):
    out = set()
    for m in re.finditer(r"v\[(\d+):(\d+)\]", text):
        out |= set(range(int(m.group(1)), int(m.group(2)) + 1))
    for m in re.finditer(r"\bv(\d+)\b", text):
        out.add(int(m.group(1)))
    return out


@pytest.fixture(scope="module", params=["rotseq_chain.hip", "rotseq_refl3.hip"])
def chain_asm(request, tmp_path_factory):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("isa") / (request.param + ".s")
    from paper_2412_01852_amd import build
    # the library's own flags, so the scanned code is the code that runs
    cmd = [HIPCC, *build.FLAGS, "--cuda-device-only", "-S",
           os.path.join(CSRC, request.param), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def test_no_valu_write_before_dpp_read(chain_asm):
    # Compiler output lines start with a tab; the lines of a multi-line
    # inline asm block after its first do not, so take every line that
    # starts with an instruction mnemonic.
    ins = [l.strip() for l in chain_asm.split("\n")
           if re.match(r"\s*(v|s|ds|buffer|global|flat|scratch)_[a-z0-9_]+(\s|$)", l)]
    ndpp = 0
    bad = []
    for i, t in enumerate(ins):
        op = t.split()[0]
        if not op.endswith("_dpp"):
            continue
        ndpp += 1
        src0 = vregs(t.split(None, 1)[1].split(",")[1])
        for j in (1, 2):
            if i - j < 0:
                break
            prev = ins[i - j]
            pop = prev.split()[0]
            if pop.startswith("v_") and not pop.startswith(("v_readfirstlane", "v_readlane", "v_cmp", "v_writelane")) \
                    and " " in prev and vregs(prev.split(None, 1)[1].split(",")[0]) & src0:
                bad.append((prev, t))
    assert ndpp > 1000, "expected DPP coefficient broadcasts in the sweep"
    assert not bad, f"{len(bad)} DPP reads follow a VALU write of their source, e.g. {bad[:2]}"


def test_no_scratch_spills(chain_asm):
    for m in re.finditer(r"\.name:\s+(\S*sweep_chain\S*)(.*?)\.vgpr_spill_count:\s+(\d+)", chain_asm, re.S):
        pass
    spills = re.findall(r"\.vgpr_spill_count:\s+(\d+)", chain_asm)
    assert spills and all(int(v) == 0 for v in spills), "VGPR spills in a sweep kernel"
    assert "private_segment_fixed_size: 0" in chain_asm.replace("  ", " ") or \
        all(int(v) == 0 for v in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", chain_asm))
