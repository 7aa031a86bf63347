"""Compiled-code check of the assembly kernels (CPU only: hipcc cross-compiles for gfx950).

A value that stays live through a divergent `if` must be spilled (to scratch, or copied to
an accumulation register) with the full exec mask: a copy made while the `if` has narrowed
exec is never written for the lanes outside it, and those lanes later reload whatever the
slot held.  That is how a corner select written as a compare chain broke the general
exponent wedge Jacobian (stale slot offsets and ranks: wrong values, varying between runs,
and out-of-range LDS/CSR addresses).  The scan below walks each kernel's code in order,
tracks the `if` regions opened by s_and_saveexec_b64 and closed by the matching exec
restore, and reports spill stores and accumulation-register writes made inside a region of
a VGPR last defined before that region opened.  A linear walk does not follow every
control-flow shape, so the scan is pinned on hand-written snippets of both patterns.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2204_04321_amd import build

_DEF_PREFIXES = ("v_", "global_load", "scratch_load", "flat_load", "buffer_load", "ds_read")


def _vregs(tok):
    m = re.match(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def masked_live_spills(asm, pattern=r"(?:owner|ensemble)_kernel"):
    """{kernel symbol: [(line, instruction)]} of spills of live-through values made under a
    narrowed exec mask."""
    out = {}
    for name in re.findall(r"^(_Z\S*" + pattern + r"\S*):", asm, re.M):
        i = asm.index("\n" + name + ":")
        j = asm.find(".Lfunc_end", i)
        lines = [l.split(";")[0].strip() for l in asm[i:(j if j > 0 else len(asm))].split("\n")]
        open_ifs, last_def, bad = [], {}, []
        for k, t in enumerate(lines):
            m = re.match(r"s_and_saveexec_b64 (s\[\d+:\d+\])", t)
            if m:
                open_ifs.append((m.group(1), k))
                continue
            m = re.match(r"s_or_b64 exec, exec, (s\[\d+:\d+\])", t)
            if m and any(r == m.group(1) for r, _ in open_ifs):
                idx = max(n for n, (r, _) in enumerate(open_ifs) if r == m.group(1))
                del open_ifs[idx:]
                continue
            parts = t.replace(",", " ").split()
            if not parts:
                continue
            op = parts[0]
            if open_ifs and (op.startswith("scratch_store") or op == "v_accvgpr_write_b32"):
                opened = open_ifs[0][1]
                if any(last_def.get(r, -1) < opened for r in _vregs(parts[2])):
                    bad.append((k, t))
            if op.startswith(_DEF_PREFIXES) and len(parts) > 1:
                for r in _vregs(parts[1]):
                    last_def[r] = k
        out[name] = bad
    return out


# a live-through value (v46, defined before the if) spilled inside the if: must be reported
_BAD = """
_Z12owner_kernelILi3ELb1EdLb0EEvv:
	v_lshrrev_b32_e32 v46, 4, v9
	v_cmp_lt_i16_e32 vcc, 0, v46
	s_and_saveexec_b64 s[0:1], vcc
	s_cbranch_execz .LBB0_2
	v_mov_b32_e32 v10, 1
.LBB0_2:
	scratch_store_dword off, v46, off offset:124 ; 4-byte Folded Spill
	v_accvgpr_write_b32 a41, v46
	s_or_b64 exec, exec, s[0:1]
	scratch_load_dword v3, off, off offset:124 ; 4-byte Folded Reload
.Lfunc_end0:
"""

# full-exec default store, then the loaded value stored inside the if; and a spill after
# the exec restore: nothing to report
_GOOD = """
_Z12owner_kernelILi3ELb1EdLb1EEvv:
	v_mov_b32_e32 v1, 0
	scratch_store_dword off, v1, off offset:120 ; 4-byte Folded Spill
	s_and_saveexec_b64 s[10:11], s[6:7]
	s_cbranch_execz .LBB1_2
	global_load_dword v2, v[2:3], off
	s_waitcnt vmcnt(0)
	scratch_store_dword off, v2, off offset:120 ; 4-byte Folded Spill
.LBB1_2:
	s_or_b64 exec, exec, s[10:11]
	v_accvgpr_write_b32 a3, v46
	scratch_store_dword off, v46, off offset:8 ; 4-byte Folded Spill
.Lfunc_end1:
"""


def test_scan_reports_masked_spill_of_live_value():
    res = masked_live_spills(_BAD)
    (hits,) = res.values()
    assert [t.split()[0] for _, t in hits] == ["scratch_store_dword", "v_accvgpr_write_b32"]
    (good,) = masked_live_spills(_GOOD).values()
    assert good == []


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_assembly_kernels_spill_live_values_with_full_exec(tmp_path):
    src = os.path.join(build.CSRC, "fo_assemble.hip")
    out = tmp_path / "fo_assemble.s"
    cmd = [build.hipcc()] + build.FLAGS + ["-x", "hip", "--cuda-device-only", "-S", src, "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    res = masked_live_spills(out.read_text())
    assert len(res) >= 20, sorted(res)            # every owner and ensemble instantiation
    bad = {k: v for k, v in res.items() if v}
    assert not bad, bad
