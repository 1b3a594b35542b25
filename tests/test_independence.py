"""The oracle and the HIP library share no code: no module of one imports the
other, the product package does not reach the oracle (no CPU fallback), and
the seeded input generators hold no method arithmetic from either side."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def sources(folder, exts=(".py",)):
    for dirpath, _, files in os.walk(os.path.join(ROOT, folder)):
        if "__pycache__" in dirpath:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(dirpath, f)


def imports(path):
    text = open(path).read()
    return set(re.findall(r"^\s*(?:from|import)\s+([A-Za-z_][\w.]*)", text, flags=re.M))


def test_oracle_does_not_import_the_product():
    for p in sources("oracle"):
        assert not any(m.startswith("paper_1612_06496_amd") for m in imports(p)), p


def test_product_does_not_import_the_oracle_or_working_files():
    for p in sources("paper_1612_06496_amd"):
        mods = imports(p)
        assert not any(m.startswith("oracle") for m in mods), p
    for p in sources("paper_1612_06496_amd", (".hip", ".hpp", ".h", ".py")):
        assert "_work" not in open(p).read(), p


def test_input_generators_import_neither_side():
    for p in sources("synth"):
        mods = imports(p)
        assert not any(m.startswith(("oracle", "paper_1612_06496_amd")) for m in mods), p
