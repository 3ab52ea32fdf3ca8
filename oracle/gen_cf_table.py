"""Write oracle/cf_nu14_oracle.json: the FP64 rounding of the high-precision
CF table computed by oracle.cf.cf_table_mp (test infrastructure)."""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle.cf import cf_table_mp, _TABLE_JSON  # noqa: E402


def main():
    tau, c, w0 = cf_table_mp()
    d = {"nu": 14, "scale": 9.0, "note": "poles with Im tau > 0, c = 2*omega",
         "tau_re": [float(t.real) for t in tau], "tau_im": [float(t.imag) for t in tau],
         "c_re": [float(x.real) for x in c], "c_im": [float(x.imag) for x in c],
         "omega0": float(w0)}
    with open(_TABLE_JSON, "w") as fh:
        json.dump(d, fh, indent=1)
    print("wrote", _TABLE_JSON)


if __name__ == "__main__":
    main()
