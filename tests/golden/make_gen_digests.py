"""Write gen_digests.json: SHA-256 digests of a few seeded generator outputs (calls only synthgen)."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import synthgen as G  # noqa: E402

rec = {
    "_about": "SHA-256 of seeded generator outputs (numpy PCG64); regenerate with make_gen_digests.py",
    "digests": {
        "image_1mib": G.digest(G.image_1mib()),
        "stream_chunk0_64k": G.digest(G.stream_chunk(0, G.stream_specs()[0], 1 << 16)),
        "xray_frame0_64k": G.digest(G.xray_frame(0, G.xray_specs(1)[0], 1 << 16)),
        "batch_specs_16": G.digest(np.array([(s.w, s.h) for s in G.batch_specs(16)], dtype=np.int64)),
    },
}
with open(os.path.join(HERE, "gen_digests.json"), "w") as f:
    json.dump(rec, f, indent=1)
    f.write("\n")
