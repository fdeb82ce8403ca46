"""Readers of the fixtures under tests/golden/ (values the paper prints, each file
citing where)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def paper_wave_cases():
    """(g, [(case, d, H / d, T / sqrt(d / g), lambda / d as printed), ...]) from
    stokes_wave_cases.txt (Sec. 7.2, Table tab_wave_cases).  The wavelength stays
    a string so that callers can see how many digits were printed."""
    g, cases = None, []
    with open(os.path.join(GOLDEN, "stokes_wave_cases.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            if line[0] == "g":
                g = float(line[1])
            else:
                name, d, h_d, t_c, lam_d, _, _ = line
                cases.append((name, float(d), float(h_d), float(t_c), lam_d))
    return g, cases
