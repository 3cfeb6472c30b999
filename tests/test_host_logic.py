"""Host-side launch logic of the batched walks, on the CPU: length classes,
the launch groups every set of present classes forms under each launch form
(one walk per wavefront, two wavefronts per walk, two or four walks per
wavefront), and the kernel-argument layout. A small program built with the
host compiler against the library's internal header prints them."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM_INCLUDE = "/opt/rocm/include"

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE),
                                reason="needs g++ and the HIP headers")

KIND_WAVE, KIND_SPLIT, KIND_GROUP2, KIND_GROUP4 = 0, 1, 2, 4


@pytest.fixture(scope="module")
def out(tmp_path_factory):
    d = tmp_path_factory.mktemp("host")
    exe = str(d / "launch_groups")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE,
                           os.path.join(ROOT, "tests", "host", "launch_groups.cpp"), "-o", exe])
    res = {"class": {}, "maxn": {}, "groups": {}}
    for line in subprocess.check_output([exe], text=True).splitlines():
        f = line.split()
        if f[0] in ("class", "maxn"):
            res[f[0]][int(f[1])] = int(f[2])
        elif f[0] == "groups":
            mask, split, lanes, n = (int(x) for x in f[1:5])
            res["groups"][(mask, split, lanes)] = [tuple(int(y) for y in x.split(":")) for x in f[5:]]
            assert len(res["groups"][(mask, split, lanes)]) == n
        else:
            res[f[0]] = int(f[1])
    return res


def test_length_classes(out):
    C = out["classes"]
    maxn = [out["maxn"][c] for c in range(C)]
    assert maxn == sorted(maxn, reverse=True) and maxn[0] == 256
    for n, c in out["class"].items():
        # the shortest class whose bound holds N
        assert n <= maxn[c] and (c == C - 1 or n > maxn[c + 1])
    # the classes the several-walks-per-wavefront kernels take: N <= 32 and N <= 16
    assert maxn[-2:] == [32, 16]
    # the two-wavefront kernel's classes: 64 < N <= 128
    assert maxn[2] == 128 and maxn[4] == 64


def test_kernel_arguments_hold_every_class(out):
    assert out["class_end_slots"] == out["classes"]
    assert out["k0_after_class_end"] == 1


@pytest.mark.parametrize("lanes", [64, 32, 16])
@pytest.mark.parametrize("split", [0, 1])
def test_launch_groups(out, split, lanes):
    C = out["classes"]
    for mask in range(1 << C):
        present = [c for c in range(C) if mask >> c & 1]
        groups = out["groups"][(mask, split, lanes)]
        covered = []
        for f, z, kind in groups:
            assert f <= z
            covered += [c for c in range(f, z + 1) if c in present]
            if kind == KIND_SPLIT:
                # the two-wavefront kernel takes both classes of 64 < N <= 128
                assert split and (f, z) == (2, 3) and (2 in present or 3 in present)
                continue
            assert f in present and z in present  # ranges start and end on present classes

            if kind == KIND_GROUP2:
                assert lanes < 64 and 6 <= f <= z <= 7 and (lanes == 32 or f == z == 6)
            elif kind == KIND_GROUP4:
                assert lanes == 16 and f == z == 7
            else:
                assert kind == KIND_WAVE
                # one layout per launch: the N > 128 classes or the shorter ones
                assert z <= 1 or f >= 2
                if split:
                    assert f >= 4 or z <= 1
                if lanes < 64:
                    assert z <= 5  # N <= 32 walks leave the one-walk-per-wavefront launch
        # every present class in exactly one launch group, in processing order
        assert covered == present
        assert [g[0] for g in groups] == sorted(g[0] for g in groups)
        assert len(groups) <= C
