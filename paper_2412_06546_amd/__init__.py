"""MI355X-native memory-saving UGKS step (arXiv:2412.06546) behind a C-ABI.

Importing the package loads nothing; `paper_2412_06546_amd.ugks` binds the
built HIP library and `paper_2412_06546_amd.cases` builds synthetic inputs.
"""
