"""Host logic of bench.py that needs no GPU: the key of the stored HBM counter
readings (the code of the library sources, comments left out), the lookup of
a reading, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

import bench


def test_code_only_drops_comments_keeps_literals():
    text = ('int a = 1; // one\n'
            '/* a block\n   comment */ const char *s = "x//y/*z*/";\n'
            "\n"
            "char q = '\"'; char r = '/';  /* t */ int b;   \n"
            "const char *e = \"esc \\\" // still a string\";\n")
    assert bench.code_only(text) == ('int a = 1;\n'
                                     'const char *s = "x//y/*z*/";\n'
                                     "char q = '\"'; char r = '/'; int b;\n"
                                     'const char *e = "esc \\" // still a string";')
    # blanks inside literals are kept as they are
    assert bench.code_only('f("a  b");   g( 1 ,\t2 );') == 'f("a  b"); g( 1 , 2 );'


def fake_tree(root, kernel_body, header="int h3d_version(void);\n"):
    os.makedirs(os.path.join(root, "paper_2307_16303_amd", "csrc"), exist_ok=True)
    os.makedirs(os.path.join(root, "include"), exist_ok=True)
    with open(os.path.join(root, "paper_2307_16303_amd", "csrc", "k.hip"), "w") as f:
        f.write(kernel_body)
    with open(os.path.join(root, "paper_2307_16303_amd", "csrc", "batch.hip"), "w") as f:
        f.write("void batch(void) {}\n")
    with open(os.path.join(root, "include", "hodlr3d.h"), "w") as f:
        f.write(header)


def test_digest_keyed_to_code_not_comments(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    fake_tree(str(tmp_path), "__global__ void k(float *p) { p[0] = 1.f; }\n")
    d0 = {s: bench.sources_digest(s) for s in ("all", "stream")}
    # a reworded or added comment keeps the key
    fake_tree(str(tmp_path), "// stage 1\n__global__ void k(float *p) { p[0] = 1.f; /* one */ }\n")
    assert {s: bench.sources_digest(s) for s in ("all", "stream")} == d0
    # a change of code changes it
    fake_tree(str(tmp_path), "__global__ void k(float *p) { p[0] = 2.f; }\n")
    assert bench.sources_digest("all") != d0["all"]
    assert bench.sources_digest("stream") != d0["stream"]
    # files of kernels launched on their own count for 'all' only
    fake_tree(str(tmp_path), "__global__ void k(float *p) { p[0] = 1.f; }\n")
    with open(os.path.join(str(tmp_path), "paper_2307_16303_amd", "csrc", "batch.hip"), "w") as f:
        f.write("void batch(int) {}\n")
    assert bench.sources_digest("stream") == d0["stream"]
    assert bench.sources_digest("all") != d0["all"]


def test_traffic_lookup(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    fake_tree(str(tmp_path), "__global__ void k(float *p) { p[0] = 1.f; }\n")
    reading = {"workload": "w", "factor_dtype": "fp32", "nrhs": 64,
               "sources_sha256": bench.sources_digest("all"), "scope": "all",
               "kernels": {"k_s1_mfma": {"fetch_kib": 1000.0, "write_kib": 10.0}}}
    monkeypatch.setattr(bench, "TRAFFIC", {"fetch_scale": 0.5, "write_scale": 1.0,
                                           "readings": [reading]})
    assert bench.traffic_bytes("k_s1_mfma", "w", "fp32", 64) == pytest.approx(
        1000.0 * 1024 / 0.5 + 10.0 * 1024)
    assert bench.traffic_bytes("k_s1_mfma", "w", "fp32", 64, adjoint=True) is None
    assert bench.traffic_bytes("k_s1_mfma", "w", "fp32", 1) is None
    assert bench.traffic_bytes("k_s2_mfma", "w", "fp32", 64) is None
    # sources changed since the reading: no figure
    fake_tree(str(tmp_path), "__global__ void k(float *p) { p[0] = 3.f; }\n")
    assert bench.traffic_bytes("k_s1_mfma", "w", "fp32", 64) is None


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.slow
@pytest.mark.parametrize("name", ["scan", "tree", "stage2_ring"])
def test_code_only_keeps_the_compiled_code(name, tmp_path):
    """A library source and its code_only text compile to the same gfx950
    device code (symbol names derived from the file path aside)."""
    import re
    import shutil
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc):
        pytest.skip("hipcc not found")
    csrc = os.path.join(bench.ROOT, "paper_2307_16303_amd", "csrc")
    (tmp_path / "include").mkdir()
    (tmp_path / "pk" / "csrc").mkdir(parents=True)
    with open(os.path.join(bench.ROOT, "include", "hodlr3d.h")) as f:
        (tmp_path / "include" / "hodlr3d.h").write_text(bench.code_only(f.read()) + "\n")
    for fn in os.listdir(csrc):
        with open(os.path.join(csrc, fn)) as f:
            (tmp_path / "pk" / "csrc" / fn).write_text(bench.code_only(f.read()) + "\n")

    def asm(src, out):
        cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang",
               "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument", "--cuda-device-only", "-S", "-o", str(out), src]
        subprocess.run(cmd, check=True, capture_output=True, timeout=600)
        keep = [ln for ln in out.read_text().split("\n")
                if not re.match(r"\s*(\.file|\.ident|;)", ln)]
        return re.sub(r"__hip_(cuid|gpubin_handle|fatbin)_[0-9a-f]+", "X", "\n".join(keep))

    a = asm(os.path.join(csrc, name + ".hip"), tmp_path / "a.s")
    b = asm(str(tmp_path / "pk" / "csrc" / (name + ".hip")), tmp_path / "b.s")
    assert "s_endpgm" in a
    assert a == b
