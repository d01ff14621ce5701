"""The device's exact-drift quotients are correctly rounded inside the
drift's window: a CPU emulation of its square-root and quotient sequences,
with the hardware estimates modelled at their measured error bounds, agrees
with the IEEE operations on several million adversarial inputs, apart from
the one family the window excludes (all-ones divisor, power-of-two
numerator).  A power-of-two drift length is therefore served by the short
sequences for every pz whose significand is not all ones, and only those
lengths need the device's significand test."""
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_drift_quotient_sequences_round_correctly(tmp_path):
    exe = str(tmp_path / "drift_quotients")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", exe,
                    os.path.join(HERE, "cpu_emulation", "drift_quotients.c"), "-lm"], check=True)
    out = subprocess.run([exe, "4000000"], check=True, capture_output=True, text=True).stdout
    m = re.search(r"sqrt misrounds (\d+); div_in (\d+) \(\+(\d+) in the excluded family\); "
                  r"div_by_root (\d+) \(\+(\d+) in the family\)", out)
    assert m, out
    sq, cur, cur_fam, new, new_fam = (int(v) for v in m.groups())
    assert sq == 0 and cur == 0 and new == 0, out
    assert cur_fam > 0 and new_fam > 0      # the excluded family is exercised
