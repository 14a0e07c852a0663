"""The guard on bench.py's committed traffic figures (no GPU needed).

bench.py reports the sweep kernel's HBM traffic from a committed counter
summary only while a hash of the kernel code matches the one the counters
were taken with.  The hash drops // comments, trailing blanks and empty
lines, so that comment edits keep the figures valid while code edits void
them; that relies on the kernel source having no block comments and no "//"
inside string literals.
"""
import importlib.util
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_kernel_source_fits_the_hash_rules():
    bench = load_bench()
    text = open(bench.KERNEL_SOURCE, encoding="utf-8").read()
    assert "/*" not in text and "*/" not in text
    for lit in re.findall(r'"(?:[^"\\\n]|\\.)*"', text):
        assert "//" not in lit, lit


def test_comment_edits_keep_the_hash_and_code_edits_change_it(tmp_path, monkeypatch):
    bench = load_bench()
    src = open(bench.KERNEL_SOURCE, encoding="utf-8").read()
    variants = {
        "same": src,
        "comment": src.replace("\n", "\n// an added comment line\n", 1) + "\n\n   \n",
        "trailing": re.sub(r"(;)\n", r"\1   // trailing note\n", src, count=5),
        "code": src.replace("0xD2511F53u", "0xD2511F55u", 1),
    }
    hashes = {}
    for name, text in variants.items():
        path = tmp_path / f"{name}.hip"
        path.write_text(text, encoding="utf-8")
        monkeypatch.setattr(bench, "KERNEL_SOURCE", str(path))
        hashes[name] = bench.kernel_code_hash()
    assert hashes["same"] == hashes["comment"] == hashes["trailing"]
    assert hashes["code"] != hashes["same"]
