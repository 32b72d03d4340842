"""CPU checks of the library: it loads, exports every entry point declared
in include/qdist.h, validates its inputs, and its host-side generator
matrices have the same structure as the oracle's (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def Q():
    from paper_2408_10743_amd import qdist
    return qdist


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "qdist.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qd_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(Q):
    names = declared_entry_points()
    assert len(names) >= 9
    lib = ctypes.CDLL(Q.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(Q.exported_symbols()) == names


def test_strerror(Q):
    for st in (0, 1, -1, -2, -3, -4, -5, -6):
        assert Q.qd_strerror(st)


def _canon(gs):
    out = []
    for g in gs:
        ins = sorted((p, d) for p, d in zip(g["pivots"], g["dims"]) if p >= 0)
        outs = sorted(d for p, d in zip(g["pivots"], g["dims"]) if p < 0)
        out.append((g["P"], g["delta"], tuple(ins), tuple(outs)))
    return out


@pytest.mark.parametrize("diag", [2, 4])
def test_structure_matches_oracle_random(Q, diag):
    for s in range(1500):
        B = W.tiny_code(70000 + s, n_max=10, m_max=20)
        if not B.any():
            continue
        assert _canon(O.gamma(B, diag, 8)) == _canon(Q.qd_plan(B, 2, diag, 8)["gammas"]), s


def test_structure_matches_oracle_configs(Q):
    for G, f in [W.config1(0), W.config2(0), W.config3(0), W.config1(5)]:
        B = O.expand(G, f)
        for diag in (2, 4):
            assert _canon(O.gamma(B, diag, 8)) == _canon(Q.qd_plan(G, f, diag, 8)["gammas"])


def test_structure_f4_input_and_wide(Q):
    for s in range(40):
        rng = W.SplitMix64(W.config_seed(30, s))
        n = rng.uniform_int(20, 128)
        if s % 2:
            G, f = W.f4_linear(n, rng.uniform_int(1, n // 2), rng.next()), 4
        else:
            G, f = W.additive(n, rng.uniform_int(1, min(2 * n, 140)), rng.next()), 2
        B = O.expand(G, f)
        for diag in (2, 4):
            assert _canon(O.gamma(B, diag, 8)) == _canon(Q.qd_plan(G, f, diag, 8)["gammas"])


def test_planner_picks_paper_structures(Q):
    # Config 2 (F4-linear [48,24]): two disjoint information sets of 24
    # two-row packages; config 3 prefers the F4 construction.
    p = Q.qd_plan(*W.config2(0))
    assert p["diag"] == 4 and p["h_used"] == 2
    assert [g["P"] for g in p["gammas"][:2]] == [24, 24]
    p3 = Q.qd_plan(*W.config3(0))
    assert p3["diag"] == 4 and p3["predicted_f4"] < p3["predicted_f2"]


def test_plan_input_validation(Q):
    with pytest.raises(Q.QdError):
        Q.qd_plan(np.zeros((2, 6), np.uint8), 2)
    with pytest.raises(Q.QdError):
        Q.qd_plan(np.full((2, 6), 3, np.uint8), 2)
    with pytest.raises(Q.QdError):
        Q.qd_plan(np.ones((2, 2 * 129), np.uint8), 2)
    with pytest.raises(Q.QdError):
        Q.qd_plan(np.ones((2, 6), np.uint8), 3)


def test_no_cpu_fallback_without_gpu(Q):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    G, f = W.config1(0)
    st, d, _ = Q.qd_distance(G, f)
    assert st == Q.QD_ERR_DEVICE and d == -1
    st, w, _, _ = Q.qd_round_min(*W.random_packages(3, 8, 1), 1)
    assert st == Q.QD_ERR_DEVICE
    assert Q.qd_round_census(*W.random_packages(3, 8, 1), 1, 5)[0] == Q.QD_ERR_DEVICE
    assert Q.qd_round_min_noalloc(*W.random_packages(3, 8, 1), 1)[0] == Q.QD_ERR_DEVICE


def test_engine_needs_gpu(Q):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert not Q.qd_engine_create()


def test_valu_mix_validation(Q):
    # an unknown mix is rejected before any device work
    assert Q.qd_valu_mix(-1)[0] == Q.QD_ERR_INVALID
    assert Q.qd_valu_mix(len(Q.QD_MIXES))[0] == Q.QD_ERR_INVALID


def _iso_sets(gs):
    return [(g["P"], g["delta"], tuple(sorted(p for p in g["pivots"] if p >= 0))) for g in gs]


def _oracle_iso_sets(B):
    r, gs = O.gamma_iso(B, 8)
    return [(r, r - k, tuple(sorted(int(c) for c in piv if c >= 0))) for k, piv, _ in gs]


def test_iso_structure_matches_oracle(Q):
    # Saved_isometry: the information sets (pivot image columns) and delta of
    # every matrix are determined by the column order, whatever the basis
    for s in range(800):
        B = W.tiny_code(72000 + s, n_max=10, m_max=20)
        if not B.any():
            continue
        assert _iso_sets(Q.qd_plan(B, 2, Q.QD_DIAG_ISO, 8)["gammas"]) == _oracle_iso_sets(B), s
    for G, f in [W.config1(0), W.config2(0), W.config3(0), W.config1(5)]:
        p = Q.qd_plan(G, f, Q.QD_DIAG_ISO, 8)
        assert p["diag"] == Q.QD_DIAG_ISO
        assert _iso_sets(p["gammas"]) == _oracle_iso_sets(O.expand(G, f))
        assert p["predicted_iso"] > 0 and all(d == 1 for g in p["gammas"] for d in g["dims"])


def test_iso_planner_prefers_cheaper_construction(Q):
    # the isometry costs more than the F4 matrices on the config shapes, so
    # the automatic choice stays with F4 there
    for G, f in [W.config1(0), W.config2(0), W.config3(0)]:
        p = Q.qd_plan(G, f)
        assert p["diag"] == Q.QD_DIAG_F4 and p["predicted_f4"] <= p["predicted_iso"]


def test_filter_option_validation(Q):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    # an unknown filter is rejected before any device work
    st, d, _, _ = Q.qd_distance_ex(W.textbook_code("[[5,1,3]]"), 2, filter=7)
    assert st == Q.QD_ERR_INVALID and d == -1


def test_partial_weight_option_validation(Q):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    for v in (2, -2, 5):
        st, d, _, _ = Q.qd_distance_ex(*W.config2(0), partial_weight=v)
        assert st == Q.QD_ERR_INVALID and d == -1, v


def test_matrix_cores_option_validation(Q):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    for v in (1, -2, 7):
        st, d, _, _ = Q.qd_distance_ex(*W.config2(0), matrix_cores=v)
        assert st == Q.QD_ERR_INVALID and d == -1, v


def test_alpha_closed_binary_input_uses_scalar_classes(Q):
    # a binary input whose span is closed under alpha is F4-linear: the F4
    # prediction counts one codeword per scalar class, as for F4 input
    G, f = W.config2(0)
    B = O.expand(G, f)
    p2, p4 = Q.qd_plan(B, 2), Q.qd_plan(G, 4)
    assert p2["f4_scalar_classes"] == p4["f4_scalar_classes"] == 1
    assert p2["predicted_f4"] == p4["predicted_f4"]
    assert Q.qd_plan(*W.config1(0))["f4_scalar_classes"] == 0
    assert Q.qd_plan(W.textbook_code("[[5,1,3]]"), 2)["f4_scalar_classes"] == 1


def test_mixed_packages_structure_matches_oracle(Q):
    """Additive config-4 codes with fewer rows than qubits and enough work:
    the planner caps two-row packages (mixed packages), and the oracle's
    construction under the same caps has the same matrices (package
    dimensions, pivots, delta) on these codes.  (The oracle starts from the
    rows as given and the library from their echelon form, so in general
    the two may pick different rows and differ in detail.)"""
    codes = W.config4(count=200)
    capped = 0
    for i in range(0, 200, 2):
        G, f = codes[i]
        p = Q.qd_plan(G, f)
        caps = [c for c in p["f4_two_row_cap"] if c >= 0]
        if not caps:
            continue
        capped += 1
        assert p["diag"] == Q.QD_DIAG_F4 and p["rank"] < p["n"]
        og = O.gamma(O.expand(G, f), O.DIAG_F4, len(caps), max2=caps)
        assert len(og) == len(caps) == p["h"]
        for j, g in enumerate(og):
            mine = p["gammas"][j]
            assert (mine["P"], mine["delta"], mine["dims"], mine["pivots"]) == \
                (g["P"], g["delta"], g["dims"], g["pivots"]), (i, j)
            assert sum(1 for d, q in zip(g["dims"], g["pivots"]) if d == 2 and q >= 0) <= caps[j]
        if capped >= 6:
            break
    assert capped >= 6


def test_mixed_packages_option_validation(Q):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    for v in (2, -2):
        st, d, _, _ = Q.qd_distance_ex(*W.config1(0), mixed_packages=v)
        assert st == Q.QD_ERR_INVALID and d == -1, v


def test_resume_rejects_foreign_points(Q):
    """A resume point whose structure hash is not the code's, or whose round
    or bound is out of range, is rejected on the host before any device
    work."""
    G, f = W.config1(0)
    n = 20
    wit = np.zeros(2 * n, dtype=np.uint8)
    for point in [(2, 0, n + 1, None, 0), (2, 0, n + 1, None, 12345), (0, 0, n + 1, None, 0),
                  (2, 0, 3, wit, 0)]:
        st, d, _, _ = Q.qd_distance_ex(G, f, resume=point)
        assert st == Q.QD_ERR_INVALID and d == -1, point


def test_binding_struct_layouts_match_header(Q, tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (a C program compiled against include/qdist.h prints them)."""
    import subprocess
    structs = [Q.qd_resume, Q.qd_options, Q.qd_round_log, Q.qd_stats, Q.qd_result, Q.qd_plan_info]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "qdist.h"', "int main(void) {"]
    for cls in structs:
        name = cls.__name__
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    c_side = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cls in structs:
        name = cls.__name__
        assert c_side[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert c_side[(name, field)] == getattr(cls, field).offset, (name, field)
