"""Static check of the gfx950 assembly (CPU only): every progress-flag store
that publishes columns to the next workgroup comes after the wait that
covers the stores of those columns.

The flag stores are relaxed device-scope stores placed after a hand-coded
`s_waitcnt vmcnt(N)`; correctness relies on the compiler keeping that
order.  The test compiles the two sweeps with the library's own flags and,
for every flag store of every sweep kernel, walks back through the
instructions before it:

- vector chain sweep (`sweep_chain*`): the nearest vector memory store or
  wait before the flag store (a `global_store_dword ... sc1`) must be an
  `s_waitcnt` with vmcnt at most the publication lag (16), and no store of
  A may lie between them;
- matrix-instruction sweep (`sweep_mfma*`): flag stores (`buffer_store_dword
  ... off ... sc1`, and the final `global_store_dword ... sc1`) come after
  the first workgroup barrier, and every later barrier is preceded, with no
  store of A in between, by an `s_waitcnt` whose vmcnt is at most the
  kernel's publication count: every wave waits for its own stores, then
  all meet, then one wave publishes in the next super-step.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_01852_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PUBLISH_LAG = 16  # chain sweep: stores allowed outstanding at a publication


def compile_asm(src, tmp_path_factory):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("isa_pub") / (src + ".s")
    from paper_2412_01852_amd import build
    cmd = [HIPCC, *build.FLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def kernels(asm, name_part):
    """{mangled name: [instruction lines]} of the kernels whose name has
    `name_part`."""
    out, cur, lines = {}, None, []
    for line in asm.splitlines():
        m = re.match(r"^(_Z\w+):", line)
        if m:
            if cur:
                out[cur] = lines
            cur, lines = (m.group(1) if name_part in m.group(1) else None), []
            continue
        if cur is not None:
            if "s_endpgm" in line:
                out[cur] = lines
                cur = None
                continue
            s = line.split(";")[0].strip()
            if s and not s.startswith("."):
                lines.append(s)
    return out


def vmcnt(line):
    m = re.search(r"vmcnt\((\d+)\)", line)
    return int(m.group(1)) if m else None


def is_a_store(line):
    return re.match(r"(buffer|global)_store_dwordx[24]\b", line) is not None


@pytest.fixture(scope="module")
def chain_asm(tmp_path_factory):
    return compile_asm("rotseq_chain.hip", tmp_path_factory)


@pytest.fixture(scope="module")
def mfma_asm(tmp_path_factory):
    return compile_asm("rotseq_mfma.hip", tmp_path_factory)


def test_chain_flag_stores_follow_their_wait(chain_asm):
    ks = kernels(chain_asm, "sweep_chain")
    assert ks, "no chain sweep kernel found"
    checked = 0
    for name, lines in ks.items():
        for i, line in enumerate(lines):
            if not re.match(r"global_store_dword\b.*\bsc1\b", line):
                continue
            j = i - 1
            while j >= 0 and not (line_is_wait := lines[j].startswith("s_waitcnt") and vmcnt(lines[j]) is not None):
                assert not is_a_store(lines[j]), f"{name}: a store of A between the wait and the flag store"
                j -= 1
            assert j >= 0, f"{name}: flag store without a preceding wait"
            assert vmcnt(lines[j]) <= PUBLISH_LAG, f"{name}: {lines[j]}"
            checked += 1
    assert checked >= 2


def mfma_publication_count(name):
    """1 + kPubWait * (vector memory operations of one super-step)."""
    m = re.search(r"sweep_mfmaILi(\d)ELi(\d)E", name)
    nb, r = int(m.group(1)), int(m.group(2))
    slots = (r + 3) // 4
    per_step = 1 + 2 * slots + 2 * nb + 2 * slots + 1
    return 1 + 2 * per_step


def test_mfma_flag_stores_follow_wait_and_barrier(mfma_asm):
    ks = kernels(mfma_asm, "sweep_mfma")
    assert len(ks) >= 7, sorted(ks)
    for name, lines in ks.items():
        bound = mfma_publication_count(name)
        flags = [i for i, l in enumerate(lines)
                 if re.match(r"buffer_store_dword\s+v\d+,\s*off\b.*\bsc1\b", l)
                 or re.match(r"global_store_dword\b.*\bsc1\b", l)]
        assert flags, f"{name}: no flag store found"
        barriers = [i for i, l in enumerate(lines) if l.startswith("s_barrier")]
        assert barriers and barriers[0] < flags[0], f"{name}: a flag store before the first barrier"
        # Every barrier after the first (which follows the LDS set-up, before
        # any store) ends a super-step: before it, with no store of A in
        # between, each wave waits for its stores (inside the branch taken
        # by publishing workgroups), so the flag stored after the barrier
        # covers them.
        for j in barriers[1:]:
            w = j - 1
            while w >= 0 and not (lines[w].startswith("s_waitcnt") and vmcnt(lines[w]) is not None):
                assert not is_a_store(lines[w]), f"{name}: store of A between the wait and the barrier"
                w -= 1
            assert w >= 0 and vmcnt(lines[w]) <= bound, f"{name}: {lines[w] if w >= 0 else 'no wait'}"
