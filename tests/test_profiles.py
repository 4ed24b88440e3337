"""The committed rocprofv3 summaries under profiles/ were taken on the
kernel sources as they are now: every summary that records a kernel source
hash matches the file it names, and every summary states the command that
made it.  (bench.py reports counter-derived figures only while the hash
matches; this keeps the summaries from going stale silently.)"""
import hashlib
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1211_1646_amd", "csrc")


def source_for(name):
    return os.path.join(CSRC, "sphere_kernels.hip" if name.startswith("sphere_") else "mpmc_kernels.hip")


def summaries():
    return sorted(f for f in os.listdir(PROFILES) if f.endswith(".md"))


@pytest.mark.parametrize("name", summaries())
def test_summary_hash_matches_source(name):
    text = open(os.path.join(PROFILES, name)).read()
    m = re.search(r"kernel source sha256/16: ([0-9a-f]{16})", text)
    if not m:
        pytest.skip("no kernel source hash recorded")
    digest = hashlib.sha256(open(source_for(name), "rb").read()).hexdigest()[:16]
    assert m.group(1) == digest, "%s was taken on another version of %s" % (name, source_for(name))


@pytest.mark.parametrize("name", summaries())
def test_summary_states_its_command(name):
    text = open(os.path.join(PROFILES, name)).read()
    assert "rocprofv3" in text or "python bench.py" in text, name
