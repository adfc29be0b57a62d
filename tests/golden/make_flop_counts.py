"""Writes flop_counts.json: the arithmetic (+, -, *, /, sqrt each one flop) that the oracle performs
per node for one 2D right-hand side and one 2D limiter evaluation, counted with its operation-
counting scalar type on the 128 x 128 dam-break workload. Calls only the oracle."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))


def counts():
    import oracle
    from paper_2208_01260_amd import inputs

    pr = inputs.c3_2d(128)
    p = oracle.params_of(pr)
    c_rhs = oracle.count_rhs(p, pr.state, pr.b, pr.bx, pr.by, 20.0, 20.0)
    c_lim = oracle.count_limit(p, pr.state, pr.b, pr.bx, pr.by)
    per = lambda c: {k: v / pr.cells for k, v in c.items()}
    tot = lambda c: sum(c[k] for k in ("add", "mul", "div", "sqrt")) / pr.cells
    return {"_note": "oracle-counted operations per node, 2D, 128x128 dam break (reflective walls)",
            "rhs_per_node": per(c_rhs), "rhs_flops_per_node": tot(c_rhs),
            "limiter_per_node": per(c_lim), "limiter_flops_per_node": tot(c_lim)}


if __name__ == "__main__":
    with open(os.path.join(HERE, "flop_counts.json"), "w") as f:
        json.dump(counts(), f, indent=1)
        f.write("\n")
