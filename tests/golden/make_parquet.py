"""Writes the Parquet fixtures of this folder with pyarrow (an independent
implementation of the Apache Parquet format) from road_fines.csv, the small
hand-worked log of the road-fines example (Sec. 3 cites the Send Fine /
Insert Fine Notification pair of that process):

  road_fines_dict_v1.parquet   dictionary-coded activities, data page v1,
                               optional (nullable) columns, two row groups
  road_fines_plain_v2.parquet  PLAIN values, data page v2, required columns,
                               string case ids

Usage: python tests/golden/make_parquet.py
"""
import os

import pyarrow as pa
import pyarrow.parquet as pq

HERE = os.path.dirname(os.path.abspath(__file__))


def rows():
    out = []
    with open(os.path.join(HERE, "road_fines.csv")) as fh:
        next(fh)
        for ln in fh:
            ln = ln.strip()
            if not ln:
                continue
            case, act, ts = [x.strip('"') for x in ln.split(",")]
            out.append((int(case), act, int(ts)))
    return out


def main():
    r = rows()
    t = pa.table({"case id": pa.array([x[0] for x in r], pa.int64()),
                  "activity": pa.array([x[1] for x in r], pa.string()),
                  "timestamp": pa.array([x[2] for x in r], pa.int64())})
    pq.write_table(t, os.path.join(HERE, "road_fines_dict_v1.parquet"), compression="NONE", use_dictionary=True,
                   data_page_version="1.0", row_group_size=6, write_statistics=True)
    schema = pa.schema([pa.field("case id", pa.string(), nullable=False),
                        pa.field("activity", pa.string(), nullable=False),
                        pa.field("timestamp", pa.int64(), nullable=False)])
    t2 = pa.table({"case id": pa.array([str(x[0]) for x in r]), "activity": pa.array([x[1] for x in r]),
                   "timestamp": pa.array([x[2] for x in r], pa.int64())}, schema=schema)
    pq.write_table(t2, os.path.join(HERE, "road_fines_plain_v2.parquet"), compression="NONE", use_dictionary=False,
                   data_page_version="2.0", write_statistics=False)


if __name__ == "__main__":
    main()
