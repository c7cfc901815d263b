"""The construction step's pick contract, on the CPU.

The construction kernel picks the next node of every ant with integer
arithmetic over 16-lane rows: quantised weights q, a row prefix scan, the
draw r = floor(U * sum q / 2^32), and the test r - exclusive < q, which must
pass in exactly one slot of an open row and in none of an exhausted row.
On the device, the chosen node and a global table row are clamped into
range, so a broken pick can only give an in-range wrong choice; it marks a
node the ant does not take, so the ant's tour is not a permutation, and the
kernel checks every tour's entry sum and sum of squares against their
closed forms modulo 2^32 (tour_checksums_ok), stopping the instance with HAC_EDEVICE.
These tests pin, without a GPU:
  * the checksum test itself, compiled for the host from the same header:
    it accepts permutations and rejects a duplicate in place of a missing
    node, also two such changes whose plain sums cancel;
  * a lane-level model of the step's arithmetic, with the DPP row
    operations spelled out (row shifts fill with zero), in two forms of
    the exclusive prefix: the kernel's (P - acc + a - q) and the form of a
    variant that was taken out after a GPU fault (the row-shifted inclusive
    prefix of the lane below).  Both give exactly one hit per open row, and
    the hit is the slot the oracle's roulette chooses for the same row and
    draw;
  * the compiled kernel: no DPP instruction of hac_kernels.hip reads a
    register written by a 32-bit multiply within the four instructions
    before it.  That pattern (a v_subrev_u32_dpp reading v_mul_hi_u32's
    result two wait states later) occurs only in the removed variant's
    assembly, and the scanner is checked to find it there.
"""

import os
import re
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_19041_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CHECK_CPP = r"""
#include "hac_internal.h"
#include <cstdio>
#include <vector>
int main() {
  int n;
  while (std::scanf("%d", &n) == 1) {
    unsigned s = 0, q = 0;  // modulo 2^32, as the kernel sums them
    for (int i = 0; i < n; ++i) {
      unsigned v;
      std::scanf("%u", &v);
      s += v;
      q += v * v;
    }
    std::printf("%d\n", hac::tour_checksums_ok(n, s, q) ? 1 : 0);
  }
  return 0;
}
"""


def test_tour_checksums(tmp_path):
    src = tmp_path / "check.cpp"
    src.write_text(CHECK_CPP)
    exe = tmp_path / "check"
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    subprocess.check_call([HIPCC, "-x", "c++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I", CSRC,
                           "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)], stderr=subprocess.DEVNULL)
    rng = np.random.default_rng(11)
    cases, want = [], []
    for n in (1, 2, 3, 5, 64, 100, 1000, 65536, 1000000):
        t = rng.permutation(n)
        cases.append(t)
        want.append(1)
        if n >= 3:
            bad = t.copy()
            bad[rng.integers(n)] = bad[rng.integers(n)] if n > 1 else bad[0]
            if len(set(bad.tolist())) < n:
                cases.append(bad)
                want.append(0)
            # a duplicate of a and a missing b, plus a duplicate of c and a
            # missing d with a + c = b + d: the plain sum cancels
            if n >= 100:
                two = t.copy()
                pos = {int(v): i for i, v in enumerate(two)}
                two[pos[10]] = 9   # 9 twice, 10 missing
                two[pos[20]] = 21  # 21 twice, 20 missing
                cases.append(two)
                want.append(0)
    inp = "".join(f"{len(c)} " + " ".join(map(str, c.tolist())) + "\n" for c in cases)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split()
    assert [int(x) for x in out] == want


# ---- lane-level model of one step (16-lane rows, S slots per lane) ----
M32 = 0xFFFFFFFF


def _row_shr(v, d):
    """DPP row_shr:d with bound_ctrl: lane u of a row reads lane u - d, or 0."""
    out = np.zeros_like(v)
    for u in range(16):
        if u - d >= 0:
            out[..., u] = v[..., u - d]
    return out


def _row_scan(v):
    for d in (1, 2, 4, 8):
        v = (v + _row_shr(v, d)) & M32
    return v


def _step_model(w_bits, open_, U, S):
    """w_bits uint32 [16*S] (slot s of lane u at u*S + s), open_ bool, U uint32.
    Returns (hits [16*S] bool for the kernel's form, hits for the variant)."""
    k = len(w_bits)
    exp = (w_bits >> 23).astype(np.int64) & 0xFF
    t = np.where(open_, 150 - exp, 10 ** 6)
    sh = int(t.min())
    q = np.zeros(k, dtype=np.int64)
    if sh < 256:
        for s in range(k):
            if open_[s]:
                m = (int(w_bits[s]) & 0x7FFFFF) | 0x800000
                v = float(m) * 2.0 ** (int(exp[s]) - 150 + sh)  # ldexp(w, sh): exact
                q[s] = max(int(np.floor(v)), 1)
    q = q.reshape(16, S)
    a = np.cumsum(q, axis=1) & M32            # in-lane prefix over the lane's slots
    acc = a[:, -1]
    P = _row_scan(acc[None, :])[0]
    tot = int(acc.sum()) & M32
    r = (int(U) * tot) >> 32
    ex_kept = (P[:, None] - acc[:, None] + a - q) & M32
    Pb = _row_shr(P[None, :], 1)[0]
    ex_var = (Pb[:, None] + a - q) & M32
    hit_k = ((r - ex_kept) & M32) < q
    hit_v = ((r - ex_var) & M32) < q
    return hit_k.reshape(-1), hit_v.reshape(-1), sh >= 256


@pytest.mark.parametrize("S,k", [(1, 10), (1, 16), (2, 20), (2, 32), (4, 40), (4, 64)])
def test_step_arithmetic_picks_exactly_the_oracles_slot(S, k):
    rng = np.random.default_rng(100 + k)
    trials = 1500
    exhausted_seen = 0
    for _ in range(trials):
        # weights over many binades (normal FP32), random visited marks
        w = (rng.random(k) * 2.0 ** rng.integers(-30, 10, size=k)).astype(np.float32)
        w = np.maximum(w, np.float32(1e-30))
        vis = rng.random(k) < rng.random()
        U = int(rng.integers(0, 1 << 32))
        w_bits = np.zeros(16 * S, dtype=np.uint32)
        w_bits[:k] = w.view(np.uint32)
        open_ = np.zeros(16 * S, dtype=bool)
        open_[:k] = ~vis
        hk, hv, exhausted = _step_model(w_bits, open_, U, S)
        assert np.array_equal(hk, hv)
        if exhausted:
            exhausted_seen += 1
            assert hk.sum() == 0
            assert oracle.select(np.arange(k), w, vis.astype(np.uint8), U) == -1
            continue
        assert hk.sum() == 1
        assert int(np.flatnonzero(hk)[0]) == oracle.select(np.arange(k), w, vis.astype(np.uint8), U)
    assert 0 < exhausted_seen < trials


# ---- the compiled kernel ----
MUL = re.compile(r"\s*(v_mul_hi_u32|v_mul_lo_u32|v_mul_hi_i32|v_mad_u64_u32)\s+(v\d+)")


def _mul_fed_dpp(asm_text):
    lines = [ln for ln in asm_text.split("\n") if ln.strip() and not ln.lstrip().startswith((";", "."))
             and not ln.rstrip().endswith(":")]
    found = []
    for i, ln in enumerate(lines):
        m = MUL.match(ln)
        if not m:
            continue
        reg = m.group(2)
        for nxt in lines[i + 1:i + 5]:
            parts = nxt.split(None, 1)
            if "_dpp" in parts[0] and len(parts) > 1 and re.search(r"\b%s\b" % reg, parts[1]):
                found.append((ln.strip(), nxt.strip()))
                break
    return found


def _asm(src_path, out_path):
    flags = ["-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, "--cuda-device-only", "-S"]
    subprocess.check_call([HIPCC, *flags, str(src_path), "-o", str(out_path)], stderr=subprocess.DEVNULL)
    return out_path.read_text()


KEPT = """      ex[s] = P - acc + a[s] - q[s];
      asm volatile("" : "+v"(ex[s]));  // kept as computed: one subtraction after r"""
VARIANT = """      ex[s] = dpp_zero<0x111>(P) + a[s] - q[s];"""


def test_no_dpp_operand_from_a_multiply_in_the_kernels(tmp_path):
    from concurrent.futures import ThreadPoolExecutor
    src = open(os.path.join(CSRC, "hac_kernels.hip")).read()
    assert src.count(KEPT) == 1
    var_src = tmp_path / "variant.hip"
    var_src.write_text(src.replace(KEPT, VARIANT))
    # both compiles at once (each is one long single-threaded device pass)
    with ThreadPoolExecutor(2) as ex:
        kept_f = ex.submit(_asm, os.path.join(CSRC, "hac_kernels.hip"), tmp_path / "kept.s")
        var_f = ex.submit(_asm, var_src, tmp_path / "variant.s")
        kept, variant = kept_f.result(), var_f.result()
    assert _mul_fed_dpp(kept) == []
    # the scanner finds the pattern in the removed variant
    found = _mul_fed_dpp(variant)
    assert found and all("v_mul_hi_u32" in a and "_dpp" in b for a, b in found)
