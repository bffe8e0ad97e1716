"""bench.py's command-line contract on the host: more than one GPU is refused
before anything touches a device, and the kernel-source fingerprint that ties
the committed counter figures to the sweep's sources is stable."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], env=env,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_world_size_above_one_is_refused():
    r = _run([], {"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_kernel_source_hash_is_deterministic_and_names_existing_sources():
    import bench
    h1 = bench.kernel_source_hash()
    h2 = bench.kernel_source_hash()
    assert h1 == h2 and len(h1) == 16
    for f in bench.KERNEL_SOURCES:
        assert os.path.isfile(os.path.join(ROOT, "paper_1905_04582_amd", "csrc", f)), f


def test_kernel_source_hash_ignores_comments_only():
    import bench
    src = {f: "int a = 1; // one\n" for f in bench.KERNEL_SOURCES}
    h = bench.kernel_source_hash(src.__getitem__)
    commented = {f: "/* block */ int a = 1;   // another\n" for f in bench.KERNEL_SOURCES}
    assert bench.kernel_source_hash(commented.__getitem__) == h
    changed = dict(src)
    changed[bench.KERNEL_SOURCES[0]] = "int a = 2; // one\n"
    assert bench.kernel_source_hash(changed.__getitem__) != h
    # comment markers inside literals are code
    assert bench.strip_comments('s = "//x"; c = \'/\';') == 's = "//x"; c = \'/\';'


def test_committed_counter_file_is_well_formed():
    # the counter figures the bench line quotes: per-form traffic, calibration
    # factor and the fingerprint of the sources they were taken on
    with open(os.path.join(ROOT, "profiles", "sweep_traffic.json")) as fh:
        t = json.load(fh)
    assert len(t["kernel_source_sha"]) == 16
    assert t["n"] == 5392
    for form in ("fp64", "fp32"):
        assert form in t
